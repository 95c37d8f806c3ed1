// Row-walk choices of the FP32 centre copy for Lloyd and Hamerly fits, per
// row-length class (0: under 48 stored entries per row on average, 1: 48
// or more).  Written by paper_2107_04074_amd/tune_walk.py on gfx950, 256 compute units,
// 20000 seeded tf-idf rows, k = 3 kp / 4, row-walk time of a Lloyd and a
// Hamerly fit of 15 steps at most (HIP events), best of the repetitions:
//   layout kp   32, mean row 24, d 20000: 0.642 ms default, 0.939 ms alternative -> 0
//   layout kp   64, mean row 24, d 20000: 0.805 ms default, 0.987 ms alternative -> 0
//   layout kp  128, mean row 24, d 20000: 1.123 ms default, 1.185 ms alternative -> 0
//   layout kp  256, mean row 24, d 20000: 1.228 ms default, 1.415 ms alternative -> 0
//   slices kp  512, mean row 24, d 10000: 3.625 ms sliced, 1.898 ms whole rows -> 0
//   slices kp 1024, mean row 24, d 10000: 4.153 ms sliced, 3.503 ms whole rows -> 0
//   slices kp 2048, mean row 24, d 10000: 7.867 ms sliced, 6.945 ms whole rows -> 0
//   slices kp 4096, mean row 24, d 10000: 13.085 ms sliced, 13.904 ms whole rows -> 1
//   layout kp   32, mean row 80, d 20000: 1.442 ms default, 1.532 ms alternative -> 0
//   layout kp   64, mean row 80, d 20000: 1.583 ms default, 1.465 ms alternative -> 1
//   layout kp  128, mean row 80, d 20000: 1.996 ms default, 2.006 ms alternative -> 0
//   layout kp  256, mean row 80, d 20000: 1.583 ms default, 1.702 ms alternative -> 0
//   slices kp  512, mean row 80, d 10000: 3.770 ms sliced, 2.413 ms whole rows -> 0
//   slices kp 1024, mean row 80, d 10000: 3.831 ms sliced, 4.535 ms whole rows -> 1
//   slices kp 2048, mean row 80, d 10000: 4.756 ms sliced, 6.621 ms whole rows -> 1
//   slices kp 4096, mean row 80, d 10000: 6.517 ms sliced, 12.887 ms whole rows -> 1
#pragma once

namespace skm {
// Layout per padded width kp = 16, 32, 64, 128, 256 (index log2(kp) - 4).
// 0: the default layout (k <= 64: a group of kp/4 lanes per row, several rows
// per wave; k in (64, 256]: one row per wave, one 16-byte unit per lane);
// 1: the alternative (k in (16, 64]: one row per wave in sub-waves of kp/4
// lanes, 64/(kp/4) stored entries per gather instruction; k in (64, 256]:
// one row per wave, two 16-byte units per lane, sub-waves of kp/8 lanes).
constexpr int kWalkTuneWidths = 5;
constexpr int kWalkTuneRowClasses = 2;
constexpr int kWalkTuneShortRow = 48;  // mean stored entries per row below: class 0
constexpr int kWalkTune[kWalkTuneRowClasses][kWalkTuneWidths] = {
    {0, 0, 0, 0, 0},
    {0, 0, 1, 0, 0}
};
// Slicing per padded width kp = 512, 1024, 2048, 4096 (index log2(kp) - 9)
// while the copy fits the last-level cache: 1 = walk 256 centres per
// launch, 0 = whole rows in one launch.
constexpr int kChunkTuneWidths = 4;
constexpr int kChunkTune[kWalkTuneRowClasses][kChunkTuneWidths] = {
    {0, 0, 0, 1},
    {0, 1, 1, 1}
};
}  // namespace skm
