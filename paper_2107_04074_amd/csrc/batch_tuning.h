// Row tiles of the batched row walk (rows per work item), per centre-copy
// width kp = 16, 32, ..., 4096 (index log2(kp) - 4).  Only the lockstep
// batched driver reads this table, and that driver is switched off, so the
// tiles have not been measured: one 256-row tile everywhere.
#pragma once

namespace skm {
constexpr int kBatchTileRows[9] = {256, 256, 256, 256, 256, 256, 256, 256, 256};
}  // namespace skm
