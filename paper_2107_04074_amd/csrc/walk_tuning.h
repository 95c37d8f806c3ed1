// Row-walk layout of the FP32 centre copy for Lloyd and Hamerly fits, per
// padded width kp = 16, 32, 64, 128, 256 (index log2(kp) - 4) and row-length
// class (0: under 48 stored entries per row on average, 1: 48 or more).
// 0: the default layout (k <= 64: a group of kp/4 lanes per row, several rows
// per wave; k in (64, 256]: one row per wave, one 16-byte unit per lane);
// 1: the alternative (k in (16, 64]: one row per wave in sub-waves of kp/4
// lanes, 64/(kp/4) stored entries per gather instruction; k in (64, 256]:
// one row per wave, two 16-byte units per lane, sub-waves of kp/8 lanes).
// Written by paper_2107_04074_amd/tune_walk.py on gfx950, 256 compute units:
// 20000 x 20000 seeded tf-idf rows, k = 3 kp / 4, row-walk time of a Lloyd and
// a Hamerly fit of 15 steps at most (HIP events), best of the repetitions:
//   kp   32, mean row 24: row walks 0.673 ms (default), 0.960 ms (alternative) -> 0
//   kp   64, mean row 24: row walks 0.798 ms (default), 0.984 ms (alternative) -> 0
//   kp  128, mean row 24: row walks 1.110 ms (default), 1.175 ms (alternative) -> 0
//   kp  256, mean row 24: row walks 1.224 ms (default), 1.417 ms (alternative) -> 0
//   kp   32, mean row 80: row walks 1.476 ms (default), 1.604 ms (alternative) -> 0
//   kp   64, mean row 80: row walks 1.541 ms (default), 1.501 ms (alternative) -> 1
//   kp  128, mean row 80: row walks 1.997 ms (default), 2.020 ms (alternative) -> 0
//   kp  256, mean row 80: row walks 1.784 ms (default), 1.953 ms (alternative) -> 0
#pragma once

namespace skm {
constexpr int kWalkTuneWidths = 5;
constexpr int kWalkTuneRowClasses = 2;
constexpr int kWalkTuneShortRow = 48;  // mean stored entries per row below: class 0
constexpr int kWalkTune[kWalkTuneRowClasses][kWalkTuneWidths] = {
    {0, 0, 0, 0, 0},
    {0, 0, 1, 0, 0}
};
}  // namespace skm
