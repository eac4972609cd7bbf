// Decoder instantiation: math float, message storage float, rule CVR_SP.
#include "cvr_decode_impl.h"

namespace cvr {
CVR_DECL_DISPATCH(decode_f32_sp)
{
    return dispatch_deg<float, float, CVR_SP>(b, a, s, qc, mode, queue, gridws, sh);
}
}  // namespace cvr
