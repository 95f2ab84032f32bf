// Landmark kernel-PCA lifting for GW_PEN_POWER and the gradient path.
#include "runtime.h"

namespace gwr {

void release_landmarks(Ctx& c) {
    for (int s = 0; s < 2; ++s) c.side[s].lm.fitted = false;
}

Status lift_nystrom(Ctx& c, int side, const float* x, int64_t n, int d, const float* w, float* X, int64_t n_pad,
                    const std::string& tag) {
    (void)c; (void)side; (void)x; (void)n; (void)d; (void)w; (void)X; (void)n_pad; (void)tag;
    return fail(GW_EUNSUPPORTED, "power penalty lifting not built yet");
}

Status Solve::gradients(float* grad_x, float* grad_a, float* grad_y, float* grad_b) {
    (void)grad_x; (void)grad_a; (void)grad_y; (void)grad_b;
    return fail(GW_EUNSUPPORTED, "gradients not built yet");
}

}  // namespace gwr
