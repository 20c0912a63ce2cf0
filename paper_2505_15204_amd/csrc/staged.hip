// staged.hip — the staged form's chunk kernels (staged.hpp) for one precision form, chosen at
// compile time by BLINK_STAGED_PREC (BLINK_PREC_FP32, _SPLIT_F16 or _SPLIT_BF16); the library
// links one object per precision.
#include "staged.hpp"

#ifndef BLINK_STAGED_PREC
#error "compile with -DBLINK_STAGED_PREC=0 (FP32), 1 (FP16) or 2 (BF16)"
#endif

namespace blink {

template struct StagedLaunch<BLINK_STAGED_PREC>;

}  // namespace blink
