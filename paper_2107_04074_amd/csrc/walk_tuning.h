// Row-walk choices of the FP32 centre copy, per row-length class (0: under
// 20 stored entries per row on average, 1: under 48, 2: more).  Written by
// paper_2107_04074_amd/tune_walk.py on gfx950, 256 compute units, 100000 seeded
// tf-idf rows, k = 3 kp / 4, summed row-walk time of one fit of every variant
// of the family (15 steps at most, HIP events), best of the repetitions:
//   layout kp   32, mean row  6, d 20000: 1.085 ms default, 3.294 ms alternative -> 0
//   layout kp   64, mean row  6, d 20000: 1.312 ms default, 3.400 ms alternative -> 0
//   layout kp  128, mean row  6, d 20000: 3.830 ms default, 1.889 ms alternative -> 1
//   layout kp  256, mean row  6, d 20000: 3.774 ms default, 3.104 ms alternative -> 1
//   layout kp  512, mean row  6, d 20000: 5.457 ms default, 6.532 ms alternative -> 0
//   slices lloyd+hamerly      kp  512, mean row  6, d 10000: 8.612 ms sliced, 4.766 ms whole rows -> 0
//   slices simp_elkan+elkan   kp  512, mean row  6, d 10000: 19.539 ms sliced, 11.785 ms whole rows -> 0
//   slices yinyang            kp  512, mean row  6, d 10000: 6.891 ms sliced, 3.183 ms whole rows -> 0
//   slices lloyd+hamerly      kp 1024, mean row  6, d 10000: 13.094 ms sliced, 8.238 ms whole rows -> 0
//   slices simp_elkan+elkan   kp 1024, mean row  6, d 10000: 42.385 ms sliced, 20.954 ms whole rows -> 0
//   slices yinyang            kp 1024, mean row  6, d 10000: 11.458 ms sliced, 4.765 ms whole rows -> 0
//   slices lloyd+hamerly      kp 2048, mean row  6, d 10000: 33.609 ms sliced, 15.418 ms whole rows -> 0
//   slices simp_elkan+elkan   kp 2048, mean row  6, d 10000: 97.106 ms sliced, 71.444 ms whole rows -> 0
//   slices yinyang            kp 2048, mean row  6, d 10000: 29.160 ms sliced, 9.264 ms whole rows -> 0
//   slices lloyd+hamerly      kp 4096, mean row  6, d 10000: 87.611 ms sliced, 37.846 ms whole rows -> 0
//   slices simp_elkan+elkan   kp 4096, mean row  6, d 10000: 209.954 ms sliced, 134.302 ms whole rows -> 0
//   slices yinyang            kp 4096, mean row  6, d 10000: 72.161 ms sliced, 25.485 ms whole rows -> 0
//   layout kp   32, mean row 30, d 20000: 1.741 ms default, 3.226 ms alternative -> 0
//   layout kp   64, mean row 30, d 20000: 2.049 ms default, 3.436 ms alternative -> 0
//   layout kp  128, mean row 30, d 20000: 4.168 ms default, 3.263 ms alternative -> 1
//   layout kp  256, mean row 30, d 20000: 4.949 ms default, 6.085 ms alternative -> 0
//   layout kp  512, mean row 30, d 20000: 9.377 ms default, 13.647 ms alternative -> 0
//   slices lloyd+hamerly      kp  512, mean row 30, d 10000: 13.068 ms sliced, 8.926 ms whole rows -> 0
//   slices simp_elkan+elkan   kp  512, mean row 30, d 10000: 23.489 ms sliced, 14.013 ms whole rows -> 0
//   slices yinyang            kp  512, mean row 30, d 10000: 8.462 ms sliced, 4.707 ms whole rows -> 0
//   slices lloyd+hamerly      kp 1024, mean row 30, d 10000: 17.603 ms sliced, 18.714 ms whole rows -> 1
//   slices simp_elkan+elkan   kp 1024, mean row 30, d 10000: 36.816 ms sliced, 26.698 ms whole rows -> 0
//   slices yinyang            kp 1024, mean row 30, d 10000: 13.234 ms sliced, 9.685 ms whole rows -> 0
//   slices lloyd+hamerly      kp 2048, mean row 30, d 10000: 31.561 ms sliced, 41.161 ms whole rows -> 1
//   slices simp_elkan+elkan   kp 2048, mean row 30, d 10000: 68.589 ms sliced, 72.548 ms whole rows -> 1
//   slices yinyang            kp 2048, mean row 30, d 10000: 24.802 ms sliced, 20.588 ms whole rows -> 0
//   slices lloyd+hamerly      kp 4096, mean row 30, d 10000: 62.462 ms sliced, 100.986 ms whole rows -> 1
//   slices simp_elkan+elkan   kp 4096, mean row 30, d 10000: 133.165 ms sliced, 149.128 ms whole rows -> 1
//   slices yinyang            kp 4096, mean row 30, d 10000: 46.714 ms sliced, 49.836 ms whole rows -> 1
//   layout kp   32, mean row 80, d 20000: 3.694 ms default, 4.501 ms alternative -> 0
//   layout kp   64, mean row 80, d 20000: 4.550 ms default, 5.102 ms alternative -> 0
//   layout kp  128, mean row 80, d 20000: 7.111 ms default, 7.846 ms alternative -> 0
//   layout kp  256, mean row 80, d 20000: 11.634 ms default, 15.755 ms alternative -> 0
//   layout kp  512, mean row 80, d 20000: 25.284 ms default, 34.085 ms alternative -> 0
//   slices lloyd+hamerly      kp  512, mean row 80, d 10000: 31.277 ms sliced, 22.717 ms whole rows -> 0
//   slices simp_elkan+elkan   kp  512, mean row 80, d 10000: 42.116 ms sliced, 25.639 ms whole rows -> 0
//   slices yinyang            kp  512, mean row 80, d 10000: 16.189 ms sliced, 11.632 ms whole rows -> 0
//   slices lloyd+hamerly      kp 1024, mean row 80, d 10000: 41.495 ms sliced, 54.546 ms whole rows -> 1
//   slices simp_elkan+elkan   kp 1024, mean row 80, d 10000: 63.605 ms sliced, 58.129 ms whole rows -> 0
//   slices yinyang            kp 1024, mean row 80, d 10000: 24.459 ms sliced, 27.502 ms whole rows -> 1
//   slices lloyd+hamerly      kp 2048, mean row 80, d 10000: 68.775 ms sliced, 131.042 ms whole rows -> 1
//   slices simp_elkan+elkan   kp 2048, mean row 80, d 10000: 104.208 ms sliced, 138.999 ms whole rows -> 1
//   slices yinyang            kp 2048, mean row 80, d 10000: 42.424 ms sliced, 65.782 ms whole rows -> 1
//   slices lloyd+hamerly      kp 4096, mean row 80, d 10000: 137.100 ms sliced, 330.301 ms whole rows -> 1
//   slices simp_elkan+elkan   kp 4096, mean row 80, d 10000: 203.343 ms sliced, 341.883 ms whole rows -> 1
//   slices yinyang            kp 4096, mean row 80, d 10000: 83.792 ms sliced, 163.930 ms whole rows -> 1
#pragma once

namespace skm {
// Layout per padded width kp = 16, 32, ..., 512 (index log2(kp) - 4) of a
// whole-row walk.  0: the default layout (k <= 64: a group of kp/4 lanes per
// row, several rows per wave; k in (64, 512]: one row per wave, in two
// sub-waves of 32 lanes at kp = 128, one 16-byte unit per lane at 256, two
// at 512); 1: the alternative (k in (16, 64]: one row per wave in sub-waves
// of kp/4 lanes, 64/(kp/4) stored entries per gather instruction; k in
// (64, 512]: a group of 16 lanes per row, four rows per wave, kp/64 16-byte
// units per lane).
constexpr int kWalkTuneWidths = 6;
constexpr int kWalkTuneRowClasses = 3;
// mean stored entries per row below which a matrix is in class 0, 1
constexpr int kWalkTuneRowBound[kWalkTuneRowClasses - 1] = {20, 48};
constexpr int kWalkTune[kWalkTuneRowClasses][kWalkTuneWidths] = {
    {0, 0, 0, 1, 1, 0},
    {0, 0, 0, 1, 0, 0},
    {0, 0, 0, 0, 0, 0}
};
// Slicing per variant family (0: Lloyd and Hamerly, 1: Elkan, 2: Yin-Yang),
// row-length class and padded width kp = 512, 1024, 2048, 4096 (index
// log2(kp) - 9) while the copy fits the last-level cache: 1 = walk 256
// centres per launch, 0 = whole rows in one launch.
constexpr int kChunkTuneFamilies = 3;
constexpr int kChunkTuneWidths = 4;
constexpr int kChunkTune[kChunkTuneFamilies][kWalkTuneRowClasses][kChunkTuneWidths] = {
    {{0, 0, 0, 0}, {0, 1, 1, 1}, {0, 1, 1, 1}},
    {{0, 0, 0, 0}, {0, 0, 1, 1}, {0, 0, 1, 1}},
    {{0, 0, 0, 0}, {0, 0, 0, 1}, {0, 1, 1, 1}}
};
}  // namespace skm
