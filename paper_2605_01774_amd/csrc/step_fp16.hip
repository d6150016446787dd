// Step and adjoint launchers for the FP16 storage form.
#include "step_kernels.h"

namespace elbm {

hipError_t launch_step_fp16(const elbm_lattice* h, const void* src, void* dst, double src_mult,
                       void* lam_rec, uint8_t* br_rec) {
    return step_u<_Float16>(h, src, dst, src_mult, lam_rec, br_rec);
}

hipError_t launch_adjoint_fp16(const elbm_lattice* h, const void* state, double src_mult,
                          const void* lam_rec, const uint8_t* br_rec, const void* adj_in,
                          void* adj_out, void* t_grad) {
    return adj_u<_Float16>(h, state, src_mult, lam_rec, br_rec, adj_in, adj_out, t_grad);
}

}  // namespace elbm
