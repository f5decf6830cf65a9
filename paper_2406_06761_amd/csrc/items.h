// Work-item descriptors shared by the planner (host, no HIP dependency) and
// the kernels, which read them from device memory.
#pragma once
#include <stdint.h>

namespace wally {

// One key switch (CtRotate) work item.  Input and output are chosen by the
// launch (KsArgs::in_sel / out_sel): 0 = buf0 + off, 1 = buf1 + off, 2 = fin + off.
struct KsItem {
  const uint64_t* key;   // [L][2][L+1][n]
  uint64_t* buf0;
  uint64_t* buf1;
  uint64_t* fin;
  const uint64_t* pt;    // plaintexts of the chunk [d_pad][L][n] (giant steps)
  const uint64_t* ctp;   // rotated query copies [g][2][L][n] (giant steps)
  uint64_t* acc;         // giant-step sums [h][2][L][n] (giant steps); sel 3 reads it
  const uint64_t* key_fold;  // fold keys [log2 B][L][2][L+1][n] (folded layout)
};

// A tile of giant items that share one plaintext chunk (consecutive items).
struct MacTile {
  uint32_t first, count;
};

struct CopyItem {
  const uint64_t* src;
  uint64_t* dst;
};

}  // namespace wally
