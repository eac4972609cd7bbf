// Decoder instantiation: math double, message storage double, rule CVR_SP.
#include "cvr_decode_impl.h"

namespace cvr {
CVR_DECL_DISPATCH(decode_f64_sp)
{
    return dispatch_deg<double, double, CVR_SP>(b, a, s, qc, mode, queue, gridws, sh);
}
}  // namespace cvr
