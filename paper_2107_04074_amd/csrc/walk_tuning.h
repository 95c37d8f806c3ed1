// Row-walk choices of the FP32 centre copy, per row-length class (0: under
// 20 stored entries per row on average, 1: under 48, 2: more).  Written by
// paper_2107_04074_amd/tune_walk.py on gfx950, 256 compute units, 100000 seeded
// tf-idf rows, k = 3 kp / 4, summed row-walk time of one fit of every variant
// of the family (15 steps at most, HIP events), best of the repetitions:
//   layout kp   32, mean row  6, d 20000: 0.949 ms default, 2.875 ms alternative -> 0
//   layout kp   64, mean row  6, d 20000: 1.064 ms default, 3.011 ms alternative -> 0
//   layout kp  128, mean row  6, d 20000: 3.121 ms default, 1.421 ms alternative -> 1
//   layout kp  256, mean row  6, d 20000: 3.190 ms default, 2.367 ms alternative -> 1
//   layout kp  512, mean row  6, d 20000: 3.776 ms default, 4.415 ms alternative -> 0
//   slices lloyd+hamerly      kp  512, mean row  6, d 10000: 6.915 ms sliced, 3.699 ms whole rows -> 0
//   slices simp_elkan+elkan   kp  512, mean row  6, d 10000: 17.882 ms sliced, 10.723 ms whole rows -> 0
//   slices yinyang            kp  512, mean row  6, d 10000: 6.155 ms sliced, 2.650 ms whole rows -> 0
//   slices lloyd+hamerly      kp 1024, mean row  6, d 10000: 10.403 ms sliced, 6.063 ms whole rows -> 0
//   slices simp_elkan+elkan   kp 1024, mean row  6, d 10000: 30.573 ms sliced, 18.593 ms whole rows -> 0
//   slices yinyang            kp 1024, mean row  6, d 10000: 9.586 ms sliced, 3.637 ms whole rows -> 0
//   slices lloyd+hamerly      kp 2048, mean row  6, d 10000: 19.332 ms sliced, 11.292 ms whole rows -> 0
//   slices simp_elkan+elkan   kp 2048, mean row  6, d 10000: 61.052 ms sliced, 66.895 ms whole rows -> 1
//   slices yinyang            kp 2048, mean row  6, d 10000: 17.755 ms sliced, 7.143 ms whole rows -> 0
//   slices lloyd+hamerly      kp 4096, mean row  6, d 10000: 38.264 ms sliced, 31.619 ms whole rows -> 0
//   slices simp_elkan+elkan   kp 4096, mean row  6, d 10000: 121.033 ms sliced, 127.725 ms whole rows -> 1
//   slices yinyang            kp 4096, mean row  6, d 10000: 34.069 ms sliced, 21.750 ms whole rows -> 0
//   layout kp   32, mean row 30, d 20000: 1.734 ms default, 3.178 ms alternative -> 0
//   layout kp   64, mean row 30, d 20000: 2.045 ms default, 3.442 ms alternative -> 0
//   layout kp  128, mean row 30, d 20000: 4.176 ms default, 3.251 ms alternative -> 1
//   layout kp  256, mean row 30, d 20000: 4.944 ms default, 6.076 ms alternative -> 0
//   layout kp  512, mean row 30, d 20000: 9.294 ms default, 13.668 ms alternative -> 0
//   slices lloyd+hamerly      kp  512, mean row 30, d 10000: 12.991 ms sliced, 8.921 ms whole rows -> 0
//   slices simp_elkan+elkan   kp  512, mean row 30, d 10000: 23.460 ms sliced, 13.995 ms whole rows -> 0
//   slices yinyang            kp  512, mean row 30, d 10000: 8.439 ms sliced, 4.681 ms whole rows -> 0
//   slices lloyd+hamerly      kp 1024, mean row 30, d 10000: 17.517 ms sliced, 18.885 ms whole rows -> 1
//   slices simp_elkan+elkan   kp 1024, mean row 30, d 10000: 36.796 ms sliced, 26.722 ms whole rows -> 0
//   slices yinyang            kp 1024, mean row 30, d 10000: 13.212 ms sliced, 9.739 ms whole rows -> 0
//   slices lloyd+hamerly      kp 2048, mean row 30, d 10000: 31.487 ms sliced, 41.061 ms whole rows -> 1
//   slices simp_elkan+elkan   kp 2048, mean row 30, d 10000: 68.401 ms sliced, 72.538 ms whole rows -> 1
//   slices yinyang            kp 2048, mean row 30, d 10000: 24.748 ms sliced, 20.570 ms whole rows -> 0
//   slices lloyd+hamerly      kp 4096, mean row 30, d 10000: 62.355 ms sliced, 100.475 ms whole rows -> 1
//   slices simp_elkan+elkan   kp 4096, mean row 30, d 10000: 132.993 ms sliced, 148.756 ms whole rows -> 1
//   slices yinyang            kp 4096, mean row 30, d 10000: 46.565 ms sliced, 49.591 ms whole rows -> 1
//   layout kp   32, mean row 80, d 20000: 3.695 ms default, 4.447 ms alternative -> 0
//   layout kp   64, mean row 80, d 20000: 4.529 ms default, 5.085 ms alternative -> 0
//   layout kp  128, mean row 80, d 20000: 7.081 ms default, 7.830 ms alternative -> 0
//   layout kp  256, mean row 80, d 20000: 11.607 ms default, 15.687 ms alternative -> 0
//   layout kp  512, mean row 80, d 20000: 25.088 ms default, 33.853 ms alternative -> 0
//   slices lloyd+hamerly      kp  512, mean row 80, d 10000: 31.199 ms sliced, 22.762 ms whole rows -> 0
//   slices simp_elkan+elkan   kp  512, mean row 80, d 10000: 42.073 ms sliced, 25.844 ms whole rows -> 0
//   slices yinyang            kp  512, mean row 80, d 10000: 16.154 ms sliced, 11.663 ms whole rows -> 0
//   slices lloyd+hamerly      kp 1024, mean row 80, d 10000: 41.452 ms sliced, 54.348 ms whole rows -> 1
//   slices simp_elkan+elkan   kp 1024, mean row 80, d 10000: 63.549 ms sliced, 58.147 ms whole rows -> 0
//   slices yinyang            kp 1024, mean row 80, d 10000: 24.293 ms sliced, 27.462 ms whole rows -> 1
//   slices lloyd+hamerly      kp 2048, mean row 80, d 10000: 69.015 ms sliced, 128.929 ms whole rows -> 1
//   slices simp_elkan+elkan   kp 2048, mean row 80, d 10000: 104.224 ms sliced, 137.540 ms whole rows -> 1
//   slices yinyang            kp 2048, mean row 80, d 10000: 42.145 ms sliced, 64.884 ms whole rows -> 1
//   slices lloyd+hamerly      kp 4096, mean row 80, d 10000: 137.565 ms sliced, 332.011 ms whole rows -> 1
//   slices simp_elkan+elkan   kp 4096, mean row 80, d 10000: 203.081 ms sliced, 341.101 ms whole rows -> 1
//   slices yinyang            kp 4096, mean row 80, d 10000: 83.312 ms sliced, 167.891 ms whole rows -> 1
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
    {{0, 0, 1, 1}, {0, 0, 1, 1}, {0, 0, 1, 1}},
    {{0, 0, 0, 0}, {0, 0, 0, 1}, {0, 1, 1, 1}}
};
}  // namespace skm
