// Decoder instantiation: math float, message storage float, rule CVR_NMS.
#include "cvr_decode_impl.h"

namespace cvr {
CVR_DECL_DISPATCH(decode_f32_nms)
{
    return dispatch_deg<float, float, CVR_NMS>(b, a, s, qc, mode, queue, gridws, sh);
}
}  // namespace cvr
