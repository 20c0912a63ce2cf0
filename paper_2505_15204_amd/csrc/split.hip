// split.hip — the split-precision (matrix-core) FFT kernels for one precision, chosen at compile
// time by BLINK_SPLIT_PREC (BLINK_PREC_SPLIT_F16 or BLINK_PREC_SPLIT_BF16); the library links one
// object per precision. The kernels are the batched ones of kernels.hpp and the persistent one of
// persistent.hpp with the radix-16 stages of split_fft.hpp.
#include "kernels.hpp"
#include "persistent.hpp"

#ifndef BLINK_SPLIT_PREC
#error "compile with -DBLINK_SPLIT_PREC=1 (FP16) or 2 (BF16)"
#endif

namespace blink {

static_assert(BLINK_SPLIT_PREC == BLINK_PREC_SPLIT_F16 || BLINK_SPLIT_PREC == BLINK_PREC_SPLIT_BF16,
              "a split precision");
template struct PrecLaunch<BLINK_SPLIT_PREC>;
template struct PersistLaunch<BLINK_SPLIT_PREC>;

}  // namespace blink
