// Internal state of a lattice handle and the kernel launchers behind the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/elbm.h"

struct elbm_lattice {
    elbm_config cfg;
    int64_t n = 0;            // nodes
    int device = 0;
    hipStream_t stream = nullptr;
    void* buf[2] = {nullptr, nullptr};
    int cur = 0;              // buffer holding the current state
    // diffusion: uniform retention tensor T (host, FP64), a device field (6 values per node,
    // node-major) or a device table of 6 values per material indexed by a per-node byte
    int t_field_mode = 0;     // 0 uniform, 1 field, 2 material table
    double T_u[6] = {0, 0, 0, 0, 0, 0};
    void* t_field = nullptr;
    const uint8_t* t_phase = nullptr;
    int nphase = 0;
    bool t_set = false;
    // velocity: 0 zero, 1 uniform, 2 field (3 planes)
    int u_mode = 0;
    double u_u[3] = {0, 0, 0};
    void* u_field = nullptr;
    // source: 0 none, 1 uniform, 2 field
    int r_mode = 0;
    double r_u = 0.0;
    void* r_field = nullptr;
    double phi_lo = 0.0, phi_hi = 0.0;
    bool pending = false;     // second source half-step of the last step not yet applied
    double src_scale = 1.0;   // source amplitude s of the next steps
    double pending_scale = 1.0;  // amplitude of the pending half-step
    bool initialized = false;
    int64_t time = 0;
    // last elbm_forward_record: sizes, workspace and the start's pending flag
    int64_t rec_steps = 0, rec_ckpt = 0;
    const void* rec_ws = nullptr;
    bool rec_pending0 = false;
    bool rec_last_kept = false;  // the recompute buffers hold the last segment's forward states
    // device scratch owned by the handle
    double* d_part = nullptr;             // reduction partials
    unsigned long long* d_cnt = nullptr;  // step counters, spread over slots (lattice.h)
    long long* d_flag = nullptr;          // first bad node (validation)
    int part_blocks = 0;
};

namespace elbm {

// Largest number of blocks of the first reduction pass (their partials are 4 doubles each).
constexpr int kMaxPartBlocks = 2048;

// Bytes per stored population value of a precision form.
int store_bytes(int precision);
// Bytes of the working precision (fields, records, adjoint).
inline int real_bytes(int precision) { return precision == ELBM_F64 ? 8 : 4; }

// All launchers enqueue on h->stream and return the launch status.
hipError_t launch_step(const elbm_lattice* h, const void* src, void* dst, double src_mult,
                       void* lam_rec, uint8_t* br_rec);
hipError_t launch_adjoint(const elbm_lattice* h, const void* state, double src_mult,
                          const void* lam_rec, const uint8_t* br_rec, const void* adj_in,
                          void* adj_out, void* t_grad);
hipError_t launch_init(const elbm_lattice* h, const double* phi0, const double* j0, void* dst);
hipError_t launch_flush_source(const elbm_lattice* h, void* buf);
hipError_t launch_init_gradient(const elbm_lattice* h, const void* adj, double* dphi0, double* dj0);
// dL/dg_i = dL/dphi for every i (the readout phi = sum_i g_i), in the working precision
hipError_t launch_fill_adjoint(const elbm_lattice* h, const double* dphi, void* adj);
hipError_t launch_get_pops(const elbm_lattice* h, double* f);
hipError_t launch_set_pops(const elbm_lattice* h, const double* f, void* dst);
hipError_t launch_moments(const elbm_lattice* h, double* phi, double* q3);
// part: 4 * h->part_blocks doubles of device scratch for the block partials
hipError_t launch_reduce(const elbm_lattice* h, double* out4_dev, double* part);
hipError_t launch_min_population(const elbm_lattice* h, double* out_dev);
hipError_t launch_stream_copy(const elbm_lattice* h, const void* src, void* dst, size_t words16);
// T of `count` tensors (count = n for a field, nphase for a material table)
hipError_t launch_tensor_field(const elbm_lattice* h, const double* d6, long long count, int is_log,
                               void* t_store, long long* bad);
// first node whose material index is >= nphase
hipError_t launch_phase_check(const elbm_lattice* h, const uint8_t* phase, int nphase, long long* bad);
hipError_t launch_velocity_field(const elbm_lattice* h, const double* u3, void* u_store,
                                 long long* bad);
hipError_t launch_source_field(const elbm_lattice* h, const double* r, void* r_store);
hipError_t launch_tensor_gradient(const elbm_lattice* h, const double* d6, int is_log,
                                  const void* t_grad, double* out6);

}  // namespace elbm
