// Decoder instantiation: math float, message storage __half, rule CVR_SP.
#include "cvr_decode_impl.h"

namespace cvr {
CVR_DECL_DISPATCH(decode_f16_sp)
{
    return dispatch_deg<float, __half, CVR_SP>(b, a, s, qc, mode, queue, gridws, sh);
}
}  // namespace cvr
