// Row-walk choices of the FP32 centre copy, per row-length class (0: under
// 48 stored entries per row on average, 1: 48 or more).  Written by
// paper_2107_04074_amd/tune_walk.py on gfx950, 256 compute units, 20000 seeded
// tf-idf rows, k = 3 kp / 4, summed row-walk time of one fit of every variant
// of the family (15 steps at most, HIP events), best of the repetitions:
//   layout kp   32, mean row 24, d 20000: 0.643 ms default, 0.932 ms alternative -> 0
//   layout kp   64, mean row 24, d 20000: 0.804 ms default, 0.985 ms alternative -> 0
//   layout kp  128, mean row 24, d 20000: 1.118 ms default, 1.180 ms alternative -> 0
//   layout kp  256, mean row 24, d 20000: 1.218 ms default, 1.418 ms alternative -> 0
//   slices lloyd+hamerly      kp  512, mean row 24, d 10000: 3.636 ms sliced, 1.891 ms whole rows -> 0
//   slices simp_elkan+elkan   kp  512, mean row 24, d 10000: 5.415 ms sliced, 2.774 ms whole rows -> 0
//   slices yinyang            kp  512, mean row 24, d 10000: 2.456 ms sliced, 1.069 ms whole rows -> 0
//   slices lloyd+hamerly      kp 1024, mean row 24, d 10000: 4.163 ms sliced, 3.497 ms whole rows -> 0
//   slices simp_elkan+elkan   kp 1024, mean row 24, d 10000: 7.376 ms sliced, 5.107 ms whole rows -> 0
//   slices yinyang            kp 1024, mean row 24, d 10000: 3.181 ms sliced, 1.834 ms whole rows -> 0
//   slices lloyd+hamerly      kp 2048, mean row 24, d 10000: 7.869 ms sliced, 6.919 ms whole rows -> 0
//   slices simp_elkan+elkan   kp 2048, mean row 24, d 10000: 14.709 ms sliced, 15.088 ms whole rows -> 1
//   slices yinyang            kp 2048, mean row 24, d 10000: 5.455 ms sliced, 3.319 ms whole rows -> 0
//   slices lloyd+hamerly      kp 4096, mean row 24, d 10000: 13.027 ms sliced, 13.872 ms whole rows -> 1
//   slices simp_elkan+elkan   kp 4096, mean row 24, d 10000: 23.958 ms sliced, 26.952 ms whole rows -> 1
//   slices yinyang            kp 4096, mean row 24, d 10000: 8.069 ms sliced, 6.687 ms whole rows -> 0
//   layout kp   32, mean row 80, d 20000: 1.445 ms default, 1.534 ms alternative -> 0
//   layout kp   64, mean row 80, d 20000: 1.611 ms default, 1.472 ms alternative -> 1
//   layout kp  128, mean row 80, d 20000: 2.001 ms default, 2.013 ms alternative -> 0
//   layout kp  256, mean row 80, d 20000: 1.577 ms default, 1.725 ms alternative -> 0
//   slices lloyd+hamerly      kp  512, mean row 80, d 10000: 3.786 ms sliced, 2.445 ms whole rows -> 0
//   slices simp_elkan+elkan   kp  512, mean row 80, d 10000: 3.918 ms sliced, 2.432 ms whole rows -> 0
//   slices yinyang            kp  512, mean row 80, d 10000: 1.964 ms sliced, 1.140 ms whole rows -> 0
//   slices lloyd+hamerly      kp 1024, mean row 80, d 10000: 3.838 ms sliced, 4.608 ms whole rows -> 1
//   slices simp_elkan+elkan   kp 1024, mean row 80, d 10000: 4.066 ms sliced, 4.175 ms whole rows -> 1
//   slices yinyang            kp 1024, mean row 80, d 10000: 2.143 ms sliced, 2.027 ms whole rows -> 0
//   slices lloyd+hamerly      kp 2048, mean row 80, d 10000: 4.754 ms sliced, 6.555 ms whole rows -> 1
//   slices simp_elkan+elkan   kp 2048, mean row 80, d 10000: 5.789 ms sliced, 6.927 ms whole rows -> 1
//   slices yinyang            kp 2048, mean row 80, d 10000: 2.437 ms sliced, 2.851 ms whole rows -> 1
//   slices lloyd+hamerly      kp 4096, mean row 80, d 10000: 6.505 ms sliced, 12.810 ms whole rows -> 1
//   slices simp_elkan+elkan   kp 4096, mean row 80, d 10000: 8.552 ms sliced, 13.900 ms whole rows -> 1
//   slices yinyang            kp 4096, mean row 80, d 10000: 3.848 ms sliced, 6.585 ms whole rows -> 1
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
// Slicing per variant family (0: Lloyd and Hamerly, 1: Elkan, 2: Yin-Yang),
// row-length class and padded width kp = 512, 1024, 2048, 4096 (index
// log2(kp) - 9) while the copy fits the last-level cache: 1 = walk 256
// centres per launch, 0 = whole rows in one launch.
constexpr int kChunkTuneFamilies = 3;
constexpr int kChunkTuneWidths = 4;
constexpr int kChunkTune[kChunkTuneFamilies][kWalkTuneRowClasses][kChunkTuneWidths] = {
    {{0, 0, 0, 1}, {0, 1, 1, 1}},
    {{0, 0, 1, 1}, {0, 1, 1, 1}},
    {{0, 0, 0, 0}, {0, 0, 1, 1}}
};
}  // namespace skm
