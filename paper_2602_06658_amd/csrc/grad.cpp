// Envelope gradients of GW_eps (Appendix B.6).
#include "runtime.h"

namespace gwr {

Status Solve::gradients(float* grad_x, float* grad_a, float* grad_y, float* grad_b) {
    (void)grad_x; (void)grad_a; (void)grad_y; (void)grad_b;
    return fail(GW_EUNSUPPORTED, "gradients not built yet");
}

}  // namespace gwr
