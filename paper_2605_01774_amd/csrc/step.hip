// Precision dispatch of the step and adjoint launchers (one translation unit per storage
// form, so that the kernel instantiations compile in parallel).
#include "internal.h"

namespace elbm {

#define ELBM_FORM_DECL(tag)                                                                    \
    hipError_t launch_step_##tag(const elbm_lattice*, const void*, void*, double, void*,         \
                                 uint8_t*);                                                     \
    hipError_t launch_adjoint_##tag(const elbm_lattice*, const void*, double, const void*,       \
                                    const uint8_t*, const void*, void*, void*);
ELBM_FORM_DECL(f64)
ELBM_FORM_DECL(f32)
ELBM_FORM_DECL(bf16)
ELBM_FORM_DECL(fp16)
#undef ELBM_FORM_DECL

hipError_t launch_step(const elbm_lattice* h, const void* src, void* dst, double src_mult,
                       void* lam_rec, uint8_t* br_rec) {
    switch (h->cfg.precision) {
        case ELBM_F64: return launch_step_f64(h, src, dst, src_mult, lam_rec, br_rec);
        case ELBM_F32: return launch_step_f32(h, src, dst, src_mult, lam_rec, br_rec);
        case ELBM_BF16: return launch_step_bf16(h, src, dst, src_mult, lam_rec, br_rec);
        default: return launch_step_fp16(h, src, dst, src_mult, lam_rec, br_rec);
    }
}

hipError_t launch_adjoint(const elbm_lattice* h, const void* state, double src_mult,
                          const void* lam_rec, const uint8_t* br_rec, const void* adj_in,
                          void* adj_out, void* t_grad) {
    switch (h->cfg.precision) {
        case ELBM_F64: return launch_adjoint_f64(h, state, src_mult, lam_rec, br_rec, adj_in, adj_out, t_grad);
        case ELBM_F32: return launch_adjoint_f32(h, state, src_mult, lam_rec, br_rec, adj_in, adj_out, t_grad);
        case ELBM_BF16: return launch_adjoint_bf16(h, state, src_mult, lam_rec, br_rec, adj_in, adj_out, t_grad);
        default: return launch_adjoint_fp16(h, state, src_mult, lam_rec, br_rec, adj_in, adj_out, t_grad);
    }
}

}  // namespace elbm
