// Decoder instantiation: math double, message storage double, rule CVR_NMS.
#include "cvr_decode_impl.h"

namespace cvr {
CVR_DECL_DISPATCH(decode_f64_nms)
{
    return dispatch_deg<double, double, CVR_NMS>(b, a, s, qc, mode, queue, gridws, sh);
}
}  // namespace cvr
