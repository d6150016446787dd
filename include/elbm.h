/*
 * elbm.h - C ABI of the MI355X (gfx950) library for the local entropic lattice Boltzmann
 * scheme for the full-tensor anisotropic advection-diffusion equation
 *     d_t phi + div(phi u) = div(D grad phi) + R
 * (Feng, Leng, Jiang, Chu, arXiv 2605.01774). Lattice units dx = dt = 1, cs^2 = 1/3. The
 * library is built once per velocity set with this same ABI: libelbm.so (D3Q19) and
 * libelbm27.so (D3Q27, the paper's 3-D lattice, Sec. 2.1). Q below is 19 or 27.
 *
 * One time step = one HIP kernel: per node, the flux/ghost split of the non-equilibrium
 * populations (Sec. 2.2), the tensorial flux relaxation with S = (I/2 + D/cs^2)^-1
 * (Sec. 2.3), the ADE-corrected entropic ghost amplitude lambda (Sec. 2.5, App. B), the
 * positivity fallback alpha (Sec. 2.6), then streaming (Sec. 2.1). Sources use the midpoint
 * splitting of Sec. 3.3.
 *
 * Conventions
 *  - Grid nx * ny * nz, node index k = (z * ny + y) * nx + x (x fastest). Every per-node
 *    array passed through this interface is a set of planes [component][z][y][x], except
 *    where an entry point says otherwise.
 *  - Populations, as exchanged with elbm_get/set_populations: Q planes in this library's
 *    velocity order (elbm_velocity_table). Inside the library's population buffers the
 *    populations are stored by row: for row r = z * ny + y, the Q runs of nx values of
 *    that row lie together ([z][y][i][x]), so one row's state is one contiguous block.
 *    The library stores pre-collision populations g_i(x, t_n) in the precision form chosen
 *    at creation, as deviations d_i = g_i - W_i phi_ref (scaled by 1/store_scale for FP16).
 *  - Symmetric tensors are 6-vectors (xx, xy, xz, yy, yz, zz).
 *  - Pointers marked "device" are HIP device pointers (e.g. torch CUDA tensors); "host"
 *    pointers are ordinary CPU memory.
 *  - Sizes: every caller-owned device buffer is passed with its size in bytes (the
 *    int64_t argument named after it, <name>_bytes). The library checks each against the
 *    bytes the call reads or writes (stated per entry point; n = nx * ny * nz, "working
 *    precision" = 8 bytes for ELBM_F64, 4 otherwise) and returns ELBM_ESHAPE, touching
 *    nothing, if it is smaller; a required buffer that is NULL is ELBM_EINVAL. Optional
 *    buffers may be NULL (their size is then ignored).
 *
 * Ownership: the caller allocates and frees every population buffer, field store, record
 * and adjoint buffer; the library never frees caller memory. The library owns the handle
 * and a small device scratch area (reduction partials, step counters, flags; about 200 KB)
 * allocated at creation.
 *
 * Streams: all work is enqueued on the stream set by elbm_set_stream (default: the null
 * stream). Calls documented as synchronous wait for that stream.
 *
 * Errors: every int-returning call returns ELBM_OK (0) or a negative ELBM_E* code and
 * never throws; elbm_last_error() gives a message for the calling thread.
 */
#ifndef ELBM_H
#define ELBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ELBM_OK 0
#define ELBM_EINVAL -1    /* bad argument: null pointer, value out of range */
#define ELBM_ESHAPE -2    /* grid size unsupported, or buffers not bound */
#define ELBM_ENOTSPD -3   /* a diffusion tensor is not symmetric positive definite */
#define ELBM_EVELOCITY -4 /* some equilibrium factor E_i(u) <= 0 (|u| too large) */
#define ELBM_EHIP -5      /* HIP runtime error (message in elbm_last_error) */
#define ELBM_ESTATE -6    /* call out of order, e.g. stepping before initialisation */

/* Precision forms (storage / arithmetic) */
#define ELBM_F64 0  /* store FP64 deviations, compute FP64 */
#define ELBM_F32 1  /* store FP32 deviations, compute FP32 */
#define ELBM_BF16 2 /* store BF16 deviations (round to nearest even), compute FP32 */
#define ELBM_FP16 3 /* store FP16 deviations (round to nearest even), compute FP32 */

/* Boundary on the two x faces (y and z are always periodic) */
#define ELBM_PERIODIC 0
#define ELBM_DIRICHLET 1 /* fixed-value planes, halfway anti-bounce-back */

/* elbm_config.flags */
#define ELBM_FLAG_SCALAR_KERNEL 1 /* always use the one-node-per-thread step kernel. By
                                     default rows of nx = 64 V W nodes (W <= 8) use the
                                     row-vector kernel (V nodes per lane), other rows the
                                     one-node-per-thread kernel; results of the two are
                                     bitwise equal. */
#define ELBM_VECTOR_WIDTH_SHIFT 4 /* (flags >> 4) & 0xF: nodes per lane V in {1, 2, 4} of
                                     the row-vector kernel; 0 = automatic */
#define ELBM_FLAG_REST_FP32 2     /* BF16 / FP16 only: the rest population is stored in FP32
                                     and takes up the rounding residuals of the 18 moving
                                     populations of its node, so the stored mass equals
                                     the computed one to FP32 rounding (in each row, run 0
                                     holds nx FP32 values, the space of two 16-bit runs, and
                                     run i >= 1 starts at element (i + 1) nx) */
#define ELBM_FLAG_STOCHASTIC_ROUNDING 4 /* BF16 / FP16 only: 16-bit stores round
                                     stochastically, with bits from a counter-based hash of
                                     (time step, node, direction); deterministic for a given
                                     run. Not available to the adjoint entry points. */

typedef struct elbm_config {
    int32_t nx, ny, nz;   /* grid; each >= 1, nx * ny * nz < 2^31 */
    int32_t precision;    /* ELBM_F64 | ELBM_F32 | ELBM_BF16 | ELBM_FP16 */
    int32_t bc_x;         /* ELBM_PERIODIC | ELBM_DIRICHLET */
    int32_t flags;        /* ELBM_FLAG_* bits, 0 by default */
    double phi_ref;       /* reference scalar of the deviation storage (e.g. background) */
    double eps;           /* positivity threshold of the fallback (Sec. 2.6), >= 0 */
    double ghost_floor;   /* tau >= 0: <Dh|Dh>_H is regularised by + tau^2 phi */
    double root_rho;      /* < 0: closed-form lambda everywhere (the paper's choice);
                             >= 0: exact entropic root (FP64) at nodes whose closed-form
                             trial populations fall below root_rho * g_eq */
    double store_scale;   /* ELBM_FP16 stores d_i / store_scale (a power of two > 0) to keep
                             deviations in the FP16 normal range. Ignored (treated as 1) by
                             the other forms (BF16 has the FP32 exponent range). */
} elbm_config;

typedef struct elbm_lattice elbm_lattice; /* opaque host handle */

/* Counters accumulated by the step kernels since the last elbm_reset_counters. */
typedef struct elbm_counters {
    uint64_t fallback_nodes; /* node updates with alpha < 1 */
    uint64_t flagged_nodes;  /* node updates that took the exact entropic root */
    uint64_t nonfinite;      /* node updates whose input populations were not finite */
    uint64_t guard_nodes;    /* node updates with lambda = 1 by the guard: phi <= 0 or a zero
                                entropic denominator (Sec. 2.5 needs g_eq > 0) */
} elbm_counters;

/* Create a lattice handle from cfg (host). Allocates the handle and a small device scratch
 * on the current device. Errors: EINVAL (bad config), EHIP. */
int elbm_create(const elbm_config* cfg, elbm_lattice** out);

/* Destroy the handle and its scratch; caller buffers are untouched. NULL is accepted. */
int elbm_destroy(elbm_lattice* h);

/* Enqueue all following work on `stream` (a hipStream_t; NULL = null stream). */
int elbm_set_stream(elbm_lattice* h, void* stream);

/* Velocity table of this library: c[Q][3] (host int32) and W[Q] (host double); pass room
 * for 27 entries. Populations are indexed in this order everywhere (rest first, then
 * opposite pairs (i, i + 1), i odd). Returns Q. */
int elbm_velocity_table(int32_t* c, double* w);

/* Bytes of one population buffer: Q values per node in the storage type of the precision
 * form (with ELBM_FLAG_REST_FP32: one FP32 and Q - 1 16-bit values per node), stored by
 * row as described under Conventions. */
int64_t elbm_population_bytes(const elbm_lattice* h);

/* Bytes of one plane of a per-node field in the working precision (8 for ELBM_F64, else 4). */
int64_t elbm_field_plane_bytes(const elbm_lattice* h);

/* Bind the two population buffers (device, at least elbm_population_bytes each, distinct,
 * not aliased, 16-byte aligned: the step kernels access up to 16 bytes per lane). Step
 * kernels read one and write the other, then swap. EINVAL for null, equal or misaligned
 * buffers, ESHAPE for short ones. */
int elbm_bind_populations(elbm_lattice* h, void* buf_a, int64_t buf_a_bytes, void* buf_b,
                          int64_t buf_b_bytes);

/* Diffusion tensor, uniform (Secs. 2.3, 2.4). d6: host, 6 doubles. D must be SPD
 * (ENOTSPD otherwise). The kernels use the retention tensor T = 2 I - S = 12 D (I + 6D)^-1,
 * which keeps the small diffusive part at full relative precision. */
int elbm_set_diffusion_uniform(elbm_lattice* h, const double* d6);

/* Diffusion tensor per node. d6: device, 6 planes of FP64 (D, or the log-diffusivity L with
 * D = expm(L) if is_log != 0; 48 n bytes). t_store: device, 6 * elbm_field_plane_bytes
 * bytes, 16-byte aligned, caller-owned, must stay alive while the lattice steps; it
 * receives T node-major (the 6 components of node k at 6 k, so the step kernel reads one
 * contiguous stream). Synchronous. On ENOTSPD, *bad_node (host, may be NULL) gets the
 * first offending node index. */
int elbm_set_diffusion_field(elbm_lattice* h, const double* d6, int64_t d6_bytes, int32_t is_log,
                             void* t_store, int64_t t_store_bytes, int64_t* bad_node);

/* Diffusion tensor per material: a table of nphase tensors and one material index per node,
 * for media made of a few materials such as the two-phase porous arrays of Sec. 4.2.2 (each
 * material's tensor maps to its own S as in Sec. 2.3). It gives the same update as
 * elbm_set_diffusion_field with D(x) = table[phase(x)], bitwise, for 1 byte per node
 * instead of 6 values. d6_table: device, 6 FP64 planes of nphase entries (component c of
 * entry p at c * nphase + p, 48 nphase bytes; D, or L with D = expm(L) if is_log != 0);
 * 1 <= nphase <= 256. phase: device, n bytes (node order x fastest), caller-owned, must
 * stay alive and keep values below nphase while the lattice steps. t_store: device,
 * 6 * nphase values of the working precision, 16-byte aligned, caller-owned; it receives
 * the table's T node-major.
 * Synchronous. ENOTSPD if some entry is not SPD (*bad gets the entry), EINVAL if some
 * phase(x) >= nphase (*bad gets the first such node); bad may be NULL. The kernels clamp an
 * index to nphase - 1, so a phase buffer changed afterwards never reads outside the table.
 * The adjoint entry points need a per-node field and reject this form (ESTATE). */
int elbm_set_diffusion_phases(elbm_lattice* h, const double* d6_table, int64_t d6_table_bytes,
                              int32_t nphase, int32_t is_log, const uint8_t* phase, int64_t phase_bytes,
                              void* t_store, int64_t t_store_bytes, int64_t* bad);

/* Velocity, uniform (host, 3 doubles) or per node (u3: device, 3 planes FP64, 24 n bytes;
 * u_store: device, 3 planes of the working precision, caller-owned, 16-byte aligned: the
 * step kernels read up to 16 bytes per lane, EINVAL otherwise). Every node must have
 * E_i(u) > 0 for all i (EVELOCITY otherwise, *bad_node as above). Changing the velocity
 * while a source half-step is pending first completes that half-step with the old
 * velocity. */
int elbm_set_velocity_uniform(elbm_lattice* h, const double* u3);
int elbm_set_velocity_field(elbm_lattice* h, const double* u3, int64_t u3_bytes, void* u_store,
                            int64_t u_store_bytes, int64_t* bad_node);

/* Volumetric source R (Sec. 3.3): uniform value, or per node (r: device, one FP64 plane;
 * r_store: device, one plane of the working precision, caller-owned, 16-byte aligned,
 * EINVAL otherwise). elbm_clear_source
 * removes it. Pending half-steps are completed first, as above. */
int elbm_set_source_uniform(elbm_lattice* h, double r);
int elbm_set_source_field(elbm_lattice* h, const double* r, int64_t r_bytes, void* r_store,
                          int64_t r_store_bytes);
int elbm_clear_source(elbm_lattice* h);

/* Time dependence of the source in the separable form R(x, t) = s(t) R(x): the following
 * steps use the amplitude s for their source, i.e. s = s(t_{n+1/2}) frozen at the midpoint
 * of step n for both half-steps of the splitting of Sec. 3.3 (default 1). A half-step
 * still pending from an earlier step keeps the amplitude it was taken with (readouts and
 * the next step add it with that amplitude). Call it before each step to follow s(t).
 * The adjoint entry points take the current amplitude for both half-steps. */
int elbm_set_source_scale(elbm_lattice* h, double s);

/* Fixed values on the x = 0 side (phi_lo) and x = nx-1 side (phi_hi) for ELBM_DIRICHLET;
 * walls sit half a cell outside those nodes. */
int elbm_set_dirichlet(elbm_lattice* h, double phi_lo, double phi_hi);

/* Initial populations g = g_eq(phi0, u) (Sec. 2.1), plus the flux lift P(j0) if j0 != NULL.
 * phi0: device, one FP64 plane; j0: device, 3 FP64 planes or NULL. Writes the current
 * buffer; time is set to 0. Requires bound buffers and velocity set (default u = 0). */
int elbm_init_equilibrium(elbm_lattice* h, const double* phi0, int64_t phi0_bytes, const double* j0,
                          int64_t j0_bytes);

/* Advance n_steps >= 0 time steps (one kernel launch each, asynchronous). */
int elbm_step(elbm_lattice* h, int64_t n_steps);

/* As elbm_step, and record per node and step the amplitude lambda used (device, working
 * precision, n_steps * n values, step s at offset s * n) and the fallback branch
 * (device uint8, n_steps * n): 255 = no fallback (alpha = 1), 254 = alpha clamped to 0,
 * otherwise the direction index whose ratio set alpha. Used by the adjoint. */
int elbm_step_record(elbm_lattice* h, int64_t n_steps, void* lambda_rec, int64_t lambda_rec_bytes,
                     uint8_t* branch_rec, int64_t branch_rec_bytes);

/* One step from an explicit buffer `src` (storage form, with its pending flag, as returned
 * by elbm_save_state) into `dst` (device, elbm_population_bytes, not aliasing src; both
 * 16-byte aligned like the bound population buffers, EINVAL otherwise), with
 * optional lambda/branch records as in elbm_step_record (n values each, may be NULL).
 * The lattice's own buffers, time and pending flag are not touched. Used to recompute the
 * forward states of an adjoint segment without copies. */
int elbm_step_buffers(elbm_lattice* h, const void* src, int64_t src_bytes, int32_t pending, void* dst,
                      int64_t dst_bytes, void* lambda_rec, int64_t lambda_rec_bytes, uint8_t* branch_rec,
                      int64_t branch_rec_bytes);

/* Macroscopic readout at the current time (Secs. 2.1, 4.2.2): phi = sum g_i and the LB
 * flux q = (I - S/2) j with j = sum c_i (g_i - g_eq_i). phi: device, one FP64 plane; q3:
 * device, 3 FP64 planes; either may be NULL. */
int elbm_read_moments(elbm_lattice* h, double* phi, int64_t phi_bytes, double* q3, int64_t q3_bytes);

/* Global sums over the grid in FP64 (synchronous): out[0] = sum phi, out[1..3] = sum q.
 * Node values are accumulated with compensated summation and combined in FP64. */
int elbm_reduce(elbm_lattice* h, double* out4);

/* The sums of elbm_reduce for callers that cannot allocate or synchronise (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the same four FP64
 * sums, bitwise, written to out4 (device, 4 doubles, 32 bytes) asynchronously on the
 * lattice's stream. It calls no allocating routine: the block partials live in a static
 * device array of 64 KiB per GPU (enough for the 2048 first-pass blocks the library ever
 * uses; ESHAPE otherwise), which every call on that GPU shares and overwrites completely.
 * Calls that overlap on one GPU (other threads, other streams) race on that array.
 * Errors: EINVAL (null handle or out4), ESHAPE (out4 too small, or buffers not bound),
 * ESTATE (not initialised, no tensor). */
int elbm_reduce_noalloc(elbm_lattice* h, double* out4, int64_t out4_bytes);

/* Smallest current population g_i over all nodes and directions, FP64, as
 * elbm_get_populations would give it (full value, pending source half-step included),
 * written to *out (host, synchronous). The positivity fallback of Sec. 2.6 keeps every
 * population at or above eps after a collision, so this is the check of that bound. NaN
 * populations are skipped (elbm_get_counters counts non-finite nodes). Errors: EINVAL for a
 * null handle or output, ESHAPE without bound buffers, ESTATE before initialisation. */
int elbm_min_population(elbm_lattice* h, double* out);

/* Bandwidth reference, not part of the method: copies the src_bytes bytes of src into dst
 * (both device, 16-byte aligned, not overlapping; src_bytes a positive multiple of 16) with
 * the step kernels' access style (16 bytes per lane, nontemporal loads and stores),
 * asynchronously on the lattice's stream. Every byte is read once and written once, like
 * every stored population in a step, so its rate is a same-run reference for the HBM
 * bandwidth the step kernels achieve (on MI355X the step kernels move their bytes at about
 * the rate of this copy). Errors: EINVAL (null handle or buffer, bad size, misalignment,
 * overlap), ESHAPE (dst_bytes below src_bytes). */
int elbm_stream_copy(elbm_lattice* h, const void* src, int64_t src_bytes, void* dst, int64_t dst_bytes);

/* Current pre-collision populations g_i(x, t_n) as FP64, full values (not deviations), in
 * this library's velocity order: f: device, Q planes (8 Q n bytes). elbm_set_populations
 * loads them (rounded to the storage form) and clears any pending source half-step. */
int elbm_get_populations(elbm_lattice* h, double* f, int64_t f_bytes);
int elbm_set_populations(elbm_lattice* h, const double* f, int64_t f_bytes);

/* Raw access to the current population buffer (device pointer, storage form) and the
 * time step counter, for checkpointing: elbm_save_state copies the current buffer into
 * dst (device, elbm_population_bytes) and returns the step counter and pending flag;
 * elbm_load_state restores them. Bitwise round trip. */
int elbm_save_state(elbm_lattice* h, void* dst, int64_t dst_bytes, int64_t* step, int32_t* pending);
int elbm_load_state(elbm_lattice* h, const void* src, int64_t src_bytes, int64_t step, int32_t pending);

/* One reverse step of the discrete adjoint (hand-written vector-Jacobian product of the
 * collide-and-stream map). state: device, the population buffer (storage form) that the
 * forward step read, as saved by elbm_save_state before that step; pending: its pending
 * flag; lambda_rec / branch_rec: that step's records (n values each); adj_in: device, Q
 * planes of the working precision, dL/dg at the next time level; adj_out: device, Q
 * planes, receives dL/dg at this time level (must not alias adj_in); t_grad: device, 6
 * values of the working precision per node, node-major like the tensor store (node k's at
 * 6 k), 16-byte aligned, incremented by dL/dT of this step (T = 2 I - S as stored by
 * elbm_set_diffusion_field; the tensor must be a per-node field). */
int elbm_adjoint_step(elbm_lattice* h, const void* state, int64_t state_bytes, int32_t pending,
                      const void* lambda_rec, int64_t lambda_rec_bytes, const uint8_t* branch_rec,
                      int64_t branch_rec_bytes, const void* adj_in, int64_t adj_in_bytes, void* adj_out,
                      int64_t adj_out_bytes, void* t_grad, int64_t t_grad_bytes);

/* Checkpointed adjoint sweep. Differentiates phi after `steps` steps (the readout of
 * elbm_read_moments) with respect to the per-node tensor and the initial state: the
 * discrete adjoint of the collide-and-stream map of Secs. 2.1-2.7, one elbm_adjoint_step per
 * step in reverse order, with the forward states recomputed from a checkpoint taken every
 * `ckpt` steps. All buffers live in one caller-owned device workspace of
 * elbm_gradient_workspace_bytes(h, steps, ckpt) bytes, 256-byte aligned:
 *   steps * n lambda records (working precision) and steps * n branch bytes,
 *   ceil(steps / ckpt) checkpoints and min(ckpt, steps) - 1 recomputed states
 *   (elbm_population_bytes each), two adjoint buffers (Q planes, working precision).
 * Same conditions as elbm_adjoint_step (per-node tensor field, closed-form amplitude, no
 * FP32-rest or stochastic-rounding storage). The source amplitude is the current one for
 * every step. elbm_gradient_workspace_bytes returns the size, or a negative error code. */
int64_t elbm_gradient_workspace_bytes(const elbm_lattice* h, int64_t steps, int64_t ckpt);

/* Forward half: `steps` steps from the current state, recording lambda and the fallback
 * branch of every node and step and writing the checkpoints into the workspace. The last
 * segment's intermediate states are written into the workspace's recompute buffers, so the
 * first elbm_gradient after it does not recompute them. Leaves the lattice at the final
 * state, as elbm_step would. */
int elbm_forward_record(elbm_lattice* h, int64_t steps, int64_t ckpt, void* workspace,
                        int64_t workspace_bytes);

/* Reverse half, after elbm_forward_record with the same steps, ckpt and workspace (ESTATE
 * otherwise). dphi_n: device, one FP64 plane, dL/dphi at the final time. t_grad: device, 6
 * values per node node-major in the working precision, 16-byte aligned, incremented by
 * dL/dT (map it with elbm_tensor_gradient). dphi0 (one FP64 plane) and dj0 (3 FP64
 * planes), both device and optional (NULL), receive dL/dphi0 and dL/dj0 of an equilibrium
 * start as in elbm_initial_gradient. The lattice's own state is not touched. It may be
 * called again after the same forward run (for another dphi_n); later calls recompute every
 * segment. */
int elbm_gradient(elbm_lattice* h, int64_t steps, int64_t ckpt, void* workspace, int64_t workspace_bytes,
                  const double* dphi_n, int64_t dphi_n_bytes, void* t_grad, int64_t t_grad_bytes,
                  double* dphi0, int64_t dphi0_bytes, double* dj0, int64_t dj0_bytes);

/* Map an accumulated dL/dT (device, 6 values per node node-major, working precision, as
 * elbm_adjoint_step accumulates it) to dL/dD (is_log = 0) or
 * dL/dL (is_log = 1) per node, as derivatives with respect to the 6 stored components.
 * d6: device, the FP64 planes given to elbm_set_diffusion_field; out6: device, 6 FP64
 * planes. */
int elbm_tensor_gradient(elbm_lattice* h, const double* d6, int64_t d6_bytes, int32_t is_log,
                         const void* t_grad, int64_t t_grad_bytes, double* out6, int64_t out6_bytes);

/* Adjoint of elbm_init_equilibrium: from adj0 (device, Q planes of the working precision,
 * dL/dg at the initial time, e.g. the adj_out of the last reverse step) compute per node
 * dL/dphi0 = sum_i W_i E_i(u) adj0_i into dphi0 (device, n FP64) and, if dj0 is not null,
 * dL/dj0 = 3 sum_i W_i c_i adj0_i into dj0 (device, 3 FP64 planes). The velocity is the one
 * currently set, as at initialisation (Sec. 2.1 equilibrium, Sec. 2.2 flux lift). */
int elbm_initial_gradient(elbm_lattice* h, const void* adj0, int64_t adj0_bytes, double* dphi0,
                          int64_t dphi0_bytes, double* dj0, int64_t dj0_bytes);

/* Step counters (synchronous read) and reset. */
int elbm_get_counters(elbm_lattice* h, elbm_counters* out);
int elbm_reset_counters(elbm_lattice* h);

/* Current time step counter (number of steps since initialisation). */
int64_t elbm_time(const elbm_lattice* h);

/* Message describing the last error on the calling thread ("" if none). */
const char* elbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ELBM_H */
