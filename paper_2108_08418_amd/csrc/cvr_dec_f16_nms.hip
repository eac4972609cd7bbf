// Decoder instantiation: math float, message storage __half, rule CVR_NMS.
#include "cvr_decode_impl.h"

namespace cvr {
CVR_DECL_DISPATCH(decode_f16_nms)
{
    return dispatch_deg<float, __half, CVR_NMS>(b, a, s, qc, mode, queue, gridws, sh);
}
}  // namespace cvr
