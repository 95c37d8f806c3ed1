// Row tiles of the batched row walk (rows per work item), per centre-copy
// width kp = 16, 32, ..., 4096 (index log2(kp) - 4).  Written by
// paper_2107_04074_amd/autotune_batched.py; see the measurements below.
#pragma once

namespace skm {
// not measured yet: one 256-row tile everywhere
constexpr int kBatchTileRows[9] = {256, 256, 256, 256, 256, 256, 256, 256, 256};
}  // namespace skm
