// Discrete adjoint of the D3Q27 free-energy LB step (placeholder).
#include "lbfe_device.h"

namespace lbfe {
size_t adjoint_aux_bytes(int prec, size_t N) { return 16 * 8 * N; }
size_t adjoint_grad_slots() { return 4; }
hipError_t launch_adj_seed(hipStream_t, int, const KP &, const Bufs &, int, const double *) { return hipErrorNotSupported; }
hipError_t launch_adj_step(hipStream_t, int, const KP &, const Bufs &, int, const void *) { return hipErrorNotSupported; }
hipError_t launch_adj_init(hipStream_t, int, const KP &, const Bufs &, int, const double *, double *) {
    return hipErrorNotSupported;
}
hipError_t launch_adj_grads(hipStream_t, const KP &, const Bufs &) { return hipErrorNotSupported; }
}  // namespace lbfe
