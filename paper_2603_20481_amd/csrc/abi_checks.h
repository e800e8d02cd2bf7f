// Argument checks shared by the C entry points (host code).
#pragma once

#include "../../include/rxphy.h"

namespace rxphy {

// The C calls take the precision as an int32_t (any value a C caller may
// pass); only these three are valid.
inline bool valid_precision(int32_t p) { return p == RXPHY_FP32 || p == RXPHY_BF16 || p == RXPHY_FP16; }

}  // namespace rxphy
