// C ABI (include/elbm.h): argument validation, state bookkeeping, launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "lattice.h"

using namespace elbm;

// Device scratch of elbm_reduce_noalloc: the block partials of one reduction (4 doubles per
// block of the first pass, at most kMaxPartBlocks blocks: 64 KiB). Each GPU the library runs
// on holds its own copy until the process ends. In host code `scratch` only names the
// symbol: its device address is resolved per device (hipGetSymbolAddress, with that device
// current) when the first lattice is created there, and only that address is passed on.
static __device__ __align__(256) double scratch[4 * kMaxPartBlocks];

namespace {

thread_local std::string g_err;

int fail(int code, const char* msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* where) {
    g_err = std::string(where) + ": " + hipGetErrorString(e);
    return ELBM_EHIP;
}

#define HIP_OK(expr, where)                          \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

bool is_pow2_positive(double s) {
    if (!(s > 0) || !std::isfinite(s)) return false;
    int e;
    double m = std::frexp(s, &e);
    return m == 0.5;
}

// Retention tensor T = 12 D (I + 6 D)^-1 of a uniform tensor, FP64 on the host; false if D is
// not symmetric positive definite.
bool host_retention(const double* d6, double* t6) {
    for (int m = 0; m < 6; ++m)
        if (!std::isfinite(d6[m])) return false;
    const double D[3][3] = {{d6[0], d6[1], d6[2]}, {d6[1], d6[3], d6[4]}, {d6[2], d6[4], d6[5]}};
    if (!(D[0][0] > 0)) return false;
    const double l10 = D[1][0] / std::sqrt(D[0][0]), l20 = D[2][0] / std::sqrt(D[0][0]);
    const double p11 = D[1][1] - l10 * l10;
    if (!(p11 > 0)) return false;
    const double l21 = (D[2][1] - l20 * l10) / std::sqrt(p11);
    if (!(D[2][2] - l20 * l20 - l21 * l21 > 0)) return false;
    double M[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) M[r][c] = (r == c ? 1.0 : 0.0) + 6.0 * D[r][c];
    const double a0 = M[1][1] * M[2][2] - M[1][2] * M[2][1];
    const double a1 = M[0][2] * M[2][1] - M[0][1] * M[2][2];
    const double a2 = M[0][1] * M[1][2] - M[0][2] * M[1][1];
    const double det = M[0][0] * a0 + M[1][0] * a1 + M[2][0] * a2;
    double R[3][3];
    R[0][0] = a0 / det;
    R[0][1] = a1 / det;
    R[0][2] = a2 / det;
    R[1][0] = (M[1][2] * M[2][0] - M[1][0] * M[2][2]) / det;
    R[1][1] = (M[0][0] * M[2][2] - M[0][2] * M[2][0]) / det;
    R[1][2] = (M[0][2] * M[1][0] - M[0][0] * M[1][2]) / det;
    R[2][0] = (M[1][0] * M[2][1] - M[1][1] * M[2][0]) / det;
    R[2][1] = (M[0][1] * M[2][0] - M[0][0] * M[2][1]) / det;
    R[2][2] = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) / det;
    double T[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) T[r][c] = D[r][0] * R[0][c] + D[r][1] * R[1][c] + D[r][2] * R[2][c];
    t6[0] = 12.0 * T[0][0];
    t6[1] = 6.0 * (T[0][1] + T[1][0]);
    t6[2] = 6.0 * (T[0][2] + T[2][0]);
    t6[3] = 12.0 * T[1][1];
    t6[4] = 6.0 * (T[1][2] + T[2][1]);
    t6[5] = 12.0 * T[2][2];
    return true;
}

bool velocity_ok(const double* u) {
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    if (!std::isfinite(uu)) return false;
    for (int i = 0; i < Q; ++i) {
        const double cu = cx(i) * u[0] + cy(i) * u[1] + cz(i) * u[2];
        if (!(1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu > 0.0)) return false;
    }
    return true;
}

int check_handle(const elbm_lattice* h) {
    if (!h) return fail(ELBM_EINVAL, "null lattice handle");
    return ELBM_OK;
}

int check_bound(const elbm_lattice* h) {
    if (!h->buf[0] || !h->buf[1]) return fail(ELBM_ESHAPE, "population buffers not bound");
    return ELBM_OK;
}

int set_device(const elbm_lattice* h) {
    HIP_OK(hipSetDevice(h->device), "hipSetDevice");
    return ELBM_OK;
}

// A caller buffer and the byte size the caller gives for it: EINVAL if it is null (unless
// optional), ESHAPE if it is smaller than the `need` bytes the call will touch.
int check_buf(const void* p, int64_t bytes, int64_t need, const char* name, bool optional = false) {
    if (!p) {
        if (optional) return ELBM_OK;
        g_err = std::string(name) + " is null";
        return ELBM_EINVAL;
    }
    if (bytes < need) {
        g_err = std::string(name) + " holds " + std::to_string(bytes) + " bytes, needs " + std::to_string(need);
        return ELBM_ESHAPE;
    }
    return ELBM_OK;
}

// Bytes of `planes` per-node planes of FP64 values, and of the working precision.
int64_t f64_planes(const elbm_lattice* h, int planes) { return int64_t(planes) * h->n * 8; }
int64_t real_planes(const elbm_lattice* h, int planes) { return int64_t(planes) * h->n * real_bytes(h->cfg.precision); }
int64_t pop_bytes(const elbm_lattice* h);

// Complete a pending source half-step (before the source or the velocity changes).
int flush_pending(elbm_lattice* h) {
    if (!h->pending) return ELBM_OK;
    if (h->r_mode != 0) HIP_OK(launch_flush_source(h, h->buf[h->cur]), "flush source");
    h->pending = false;
    return ELBM_OK;
}

// Validation result of a field kernel: first offending node, or -1.
int read_flag(elbm_lattice* h, int64_t* bad_node) {
    long long v = 0;
    HIP_OK(hipMemcpyAsync(&v, h->d_flag, sizeof(v), hipMemcpyDeviceToHost, h->stream), "read flag");
    HIP_OK(hipStreamSynchronize(h->stream), "sync");
    const bool bad = v != (long long)0x7FFFFFFFFFFFFFFFLL;
    if (bad_node) *bad_node = bad ? v : -1;
    return bad ? 1 : 0;
}

int reset_flag(elbm_lattice* h) {
    // static storage: the asynchronous copy may read the host value after this returns
    static const long long kInit = 0x7FFFFFFFFFFFFFFFLL;
    HIP_OK(hipMemcpyAsync(h->d_flag, &kInit, sizeof(kInit), hipMemcpyHostToDevice, h->stream), "reset flag");
    return ELBM_OK;
}

// Conditions shared by the adjoint entry points.
int adjoint_ready(elbm_lattice* h) {
    if (h->cfg.flags & (ELBM_FLAG_REST_FP32 | ELBM_FLAG_STOCHASTIC_ROUNDING))
        return fail(ELBM_EINVAL, "the adjoint entry points do not take rest-in-FP32 or stochastic-rounding storage");
    if (!h->t_set) return fail(ELBM_ESTATE, "diffusion tensor not set");
    if (h->t_field_mode == 2) return fail(ELBM_ESTATE, "the adjoint needs a per-node tensor field, not a material table");
    if (h->cfg.root_rho >= 0) return fail(ELBM_ESTATE, "the adjoint supports the closed-form amplitude only (root_rho < 0)");
    return ELBM_OK;
}

// source multiplier of a step that starts with the given pending flag (the current
// amplitude for both half-steps, as in elbm_step_buffers)
double replay_mult(const elbm_lattice* h, bool pending) {
    return ((pending && h->r_mode != 0) ? 1.0 : 0.5) * h->src_scale;
}

// Workspace of the checkpointed sweep, each part 256-byte aligned: lambda records, branch
// records, ceil(steps / ckpt) checkpoints, ckpt - 1 recomputed states, two adjoint buffers.
struct SweepLayout {
    size_t lam, br, ck, seg, adj, adj_bytes, pop, total;
    int64_t nck;
};
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
SweepLayout sweep_layout(const elbm_lattice* h, int64_t steps, int64_t ckpt) {
    SweepLayout L{};
    const size_t n = size_t(h->n), rb = size_t(real_bytes(h->cfg.precision));
    const int64_t K = ckpt < steps ? ckpt : steps;
    L.pop = align256(size_t(elbm_population_bytes(h)));
    L.nck = (steps + ckpt - 1) / ckpt;
    L.lam = 0;
    L.br = align256(size_t(steps) * n * rb);
    L.ck = L.br + align256(size_t(steps) * n);
    L.seg = L.ck + size_t(L.nck) * L.pop;
    L.adj = L.seg + size_t(K - 1) * L.pop;
    L.adj_bytes = align256(size_t(Q) * n * rb);
    L.total = L.adj + 2 * L.adj_bytes;
    return L;
}

int64_t pop_bytes(const elbm_lattice* h) {
    if (h->cfg.flags & ELBM_FLAG_REST_FP32) return h->n * (4 + int64_t(Q - 1) * 2);
    return int64_t(Q) * h->n * store_bytes(h->cfg.precision);
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Resolve the current device's copy of `scratch` (once per device; `device` must be current).
int resolve_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(ELBM_EINVAL, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void* p = nullptr;
        HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        g_scratch_dev[device] = p;
    }
    return ELBM_OK;
}

void* scratch_of(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return (device >= 0 && device < kMaxDevices) ? g_scratch_dev[device] : nullptr;
}

}  // namespace

extern "C" {

const char* elbm_last_error(void) { return g_err.c_str(); }

int elbm_velocity_table(int32_t* c, double* w) {
    if (!c || !w) return fail(ELBM_EINVAL, "null output");
    for (int i = 0; i < Q; ++i) {
        c[3 * i + 0] = cx(i);
        c[3 * i + 1] = cy(i);
        c[3 * i + 2] = cz(i);
        w[i] = weight(i);
    }
    return Q;
}

int elbm_create(const elbm_config* cfg, elbm_lattice** out) {
    if (!cfg || !out) return fail(ELBM_EINVAL, "null argument");
    *out = nullptr;
    if (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1) return fail(ELBM_EINVAL, "grid sizes must be >= 1");
    const long long n = (long long)cfg->nx * cfg->ny * cfg->nz;
    if (n >= (1LL << 31)) return fail(ELBM_EINVAL, "nx * ny * nz must be < 2^31");
    if (cfg->precision < ELBM_F64 || cfg->precision > ELBM_FP16) return fail(ELBM_EINVAL, "bad precision");
    if (cfg->bc_x != ELBM_PERIODIC && cfg->bc_x != ELBM_DIRICHLET) return fail(ELBM_EINVAL, "bad bc_x");
    if (cfg->flags & ~(ELBM_FLAG_SCALAR_KERNEL | ELBM_FLAG_REST_FP32 | ELBM_FLAG_STOCHASTIC_ROUNDING |
                       (0xF << ELBM_VECTOR_WIDTH_SHIFT)))
        return fail(ELBM_EINVAL, "unknown flag bits");
    if ((cfg->flags & (ELBM_FLAG_REST_FP32 | ELBM_FLAG_STOCHASTIC_ROUNDING)) &&
        cfg->precision != ELBM_BF16 && cfg->precision != ELBM_FP16)
        return fail(ELBM_EINVAL, "rest-in-FP32 and stochastic rounding apply to the 16-bit forms only");
    {
        const int vw = (cfg->flags >> ELBM_VECTOR_WIDTH_SHIFT) & 0xF;
        if (vw != 0 && vw != 1 && vw != 2 && vw != 4) return fail(ELBM_EINVAL, "vector width must be 0, 1, 2 or 4");
    }
    if (!(cfg->eps >= 0) || !std::isfinite(cfg->eps)) return fail(ELBM_EINVAL, "eps must be >= 0");
    if (!(cfg->ghost_floor >= 0) || !std::isfinite(cfg->ghost_floor)) return fail(ELBM_EINVAL, "ghost_floor must be >= 0");
    if (!std::isfinite(cfg->phi_ref) || !std::isfinite(cfg->root_rho)) return fail(ELBM_EINVAL, "non-finite parameter");
    const bool scaled = cfg->precision == ELBM_FP16;
    if (scaled && !is_pow2_positive(cfg->store_scale)) return fail(ELBM_EINVAL, "store_scale must be a positive power of two");
    elbm_lattice* h = new (std::nothrow) elbm_lattice();
    if (!h) return fail(ELBM_EINVAL, "out of host memory");
    h->cfg = *cfg;
    if (!scaled) h->cfg.store_scale = 1.0;
    h->n = n;
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "hipGetDevice");
    }
    if (int r = resolve_scratch(h->device)) {
        delete h;
        return r;
    }
    long long nb = (n + 255) / 256;
    h->part_blocks = int(nb < kMaxPartBlocks ? nb : kMaxPartBlocks);
    if (h->part_blocks < 1) h->part_blocks = 1;
    const size_t bytes = sizeof(double) * (4 * (size_t)h->part_blocks + 8) + kCntWords * sizeof(unsigned long long) +
                         sizeof(long long);
    void* scratch = nullptr;
    e = hipMalloc(&scratch, bytes);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "hipMalloc scratch");
    }
    h->d_part = static_cast<double*>(scratch);
    h->d_cnt = reinterpret_cast<unsigned long long*>(h->d_part + 4 * h->part_blocks + 8);
    h->d_flag = reinterpret_cast<long long*>(h->d_cnt + kCntWords);
    e = hipMemset(h->d_cnt, 0, kCntWords * sizeof(unsigned long long));
    if (e != hipSuccess) {
        (void)hipFree(scratch);
        delete h;
        return hip_fail(e, "hipMemset");
    }
    // default tensor: none set (stepping requires one); default velocity zero
    *out = h;
    return ELBM_OK;
}

int elbm_destroy(elbm_lattice* h) {
    if (!h) return ELBM_OK;
    (void)hipSetDevice(h->device);
    if (h->d_part) (void)hipFree(h->d_part);
    delete h;
    return ELBM_OK;
}

int elbm_set_stream(elbm_lattice* h, void* stream) {
    if (int r = check_handle(h)) return r;
    h->stream = static_cast<hipStream_t>(stream);
    return ELBM_OK;
}

int64_t elbm_population_bytes(const elbm_lattice* h) {
    if (!h) return fail(ELBM_EINVAL, "null lattice handle");
    return pop_bytes(h);
}

int64_t elbm_field_plane_bytes(const elbm_lattice* h) {
    if (!h) return fail(ELBM_EINVAL, "null lattice handle");
    return h->n * real_bytes(h->cfg.precision);
}

int elbm_bind_populations(elbm_lattice* h, void* a, int64_t a_bytes, void* b, int64_t b_bytes) {
    if (int r = check_handle(h)) return r;
    if (!a || !b || a == b) return fail(ELBM_EINVAL, "need two distinct device buffers");
    if (int r = check_buf(a, a_bytes, pop_bytes(h), "buf_a")) return r;
    if (int r = check_buf(b, b_bytes, pop_bytes(h), "buf_b")) return r;
    if (reinterpret_cast<uintptr_t>(a) % 16 != 0 || reinterpret_cast<uintptr_t>(b) % 16 != 0)
        return fail(ELBM_EINVAL, "population buffers must be 16-byte aligned");
    h->buf[0] = a;
    h->buf[1] = b;
    h->cur = 0;
    h->initialized = false;
    return ELBM_OK;
}

int elbm_set_diffusion_uniform(elbm_lattice* h, const double* d6) {
    if (int r = check_handle(h)) return r;
    if (!d6) return fail(ELBM_EINVAL, "null tensor");
    double t6[6];
    if (!host_retention(d6, t6)) return fail(ELBM_ENOTSPD, "diffusion tensor is not SPD");
    for (int m = 0; m < 6; ++m) h->T_u[m] = t6[m];
    h->t_field_mode = 0;
    h->t_field = nullptr;
    h->t_phase = nullptr;
    h->nphase = 0;
    h->t_set = true;
    return ELBM_OK;
}

int elbm_set_diffusion_field(elbm_lattice* h, const double* d6, int64_t d6_bytes, int32_t is_log,
                             void* t_store, int64_t t_store_bytes, int64_t* bad_node) {
    if (int r = check_handle(h)) return r;
    if (int r = check_buf(d6, d6_bytes, f64_planes(h, 6), "d6")) return r;
    if (int r = check_buf(t_store, t_store_bytes, real_planes(h, 6), "t_store")) return r;
    if (reinterpret_cast<uintptr_t>(t_store) % 16 != 0) return fail(ELBM_EINVAL, "t_store must be 16-byte aligned");
    if (int r = set_device(h)) return r;
    if (int r = reset_flag(h)) return r;
    HIP_OK(launch_tensor_field(h, d6, h->n, is_log ? 1 : 0, t_store, h->d_flag), "tensor field");
    const int bad = read_flag(h, bad_node);
    if (bad < 0) return bad;
    if (bad) return fail(ELBM_ENOTSPD, "diffusion tensor field is not SPD at some node");
    h->t_field_mode = 1;
    h->t_field = t_store;
    h->t_phase = nullptr;
    h->nphase = 0;
    h->t_set = true;
    return ELBM_OK;
}

int elbm_set_diffusion_phases(elbm_lattice* h, const double* d6_table, int64_t table_bytes, int32_t nphase,
                              int32_t is_log, const uint8_t* phase, int64_t phase_bytes, void* t_store,
                              int64_t t_store_bytes, int64_t* bad) {
    if (int r = check_handle(h)) return r;
    if (bad) *bad = -1;
    if (nphase < 1 || nphase > 256) return fail(ELBM_EINVAL, "nphase must be in [1, 256]");
    if (int r = check_buf(d6_table, table_bytes, int64_t(6) * nphase * 8, "d6_table")) return r;
    if (int r = check_buf(phase, phase_bytes, h->n, "phase")) return r;
    if (int r = check_buf(t_store, t_store_bytes, int64_t(6) * nphase * real_bytes(h->cfg.precision), "t_store"))
        return r;
    if (reinterpret_cast<uintptr_t>(t_store) % 16 != 0) return fail(ELBM_EINVAL, "t_store must be 16-byte aligned");
    if (int r = set_device(h)) return r;
    if (int r = reset_flag(h)) return r;
    HIP_OK(launch_tensor_field(h, d6_table, nphase, is_log ? 1 : 0, t_store, h->d_flag), "tensor table");
    int b = read_flag(h, bad);
    if (b < 0) return b;
    if (b) return fail(ELBM_ENOTSPD, "diffusion tensor table is not SPD at some entry");
    if (int r = reset_flag(h)) return r;
    HIP_OK(launch_phase_check(h, phase, nphase, h->d_flag), "material index check");
    b = read_flag(h, bad);
    if (b < 0) return b;
    if (b) return fail(ELBM_EINVAL, "material index >= nphase at some node");
    h->t_field_mode = 2;
    h->t_field = t_store;
    h->t_phase = phase;
    h->nphase = nphase;
    h->t_set = true;
    return ELBM_OK;
}

int elbm_set_velocity_uniform(elbm_lattice* h, const double* u3) {
    if (int r = check_handle(h)) return r;
    if (!u3) return fail(ELBM_EINVAL, "null velocity");
    if (!velocity_ok(u3)) return fail(ELBM_EVELOCITY, "E_i(u) <= 0 for some direction");
    if (int r = set_device(h)) return r;
    if (int r = flush_pending(h)) return r;
    const bool zero = u3[0] == 0.0 && u3[1] == 0.0 && u3[2] == 0.0;
    h->u_mode = zero ? 0 : 1;
    for (int m = 0; m < 3; ++m) h->u_u[m] = zero ? 0.0 : u3[m];
    h->u_field = nullptr;
    return ELBM_OK;
}

int elbm_set_velocity_field(elbm_lattice* h, const double* u3, int64_t u3_bytes, void* u_store,
                            int64_t u_store_bytes, int64_t* bad_node) {
    if (int r = check_handle(h)) return r;
    if (int r = check_buf(u3, u3_bytes, f64_planes(h, 3), "u3")) return r;
    if (int r = check_buf(u_store, u_store_bytes, real_planes(h, 3), "u_store")) return r;
    if (reinterpret_cast<uintptr_t>(u_store) % 16 != 0) return fail(ELBM_EINVAL, "u_store must be 16-byte aligned");
    if (int r = set_device(h)) return r;
    if (int r = reset_flag(h)) return r;
    HIP_OK(launch_velocity_field(h, u3, u_store, h->d_flag), "velocity field");
    const int bad = read_flag(h, bad_node);
    if (bad < 0) return bad;
    if (bad) return fail(ELBM_EVELOCITY, "E_i(u) <= 0 at some node");
    if (int r = flush_pending(h)) return r;
    h->u_mode = 2;
    h->u_field = u_store;
    return ELBM_OK;
}

int elbm_set_source_uniform(elbm_lattice* h, double r) {
    if (int rc = check_handle(h)) return rc;
    if (!std::isfinite(r)) return fail(ELBM_EINVAL, "non-finite source");
    if (int rc = set_device(h)) return rc;
    if (int rc = flush_pending(h)) return rc;
    h->r_mode = 1;
    h->r_u = r;
    h->r_field = nullptr;
    return ELBM_OK;
}

int elbm_set_source_field(elbm_lattice* h, const double* r, int64_t r_bytes, void* r_store,
                          int64_t r_store_bytes) {
    if (int rc = check_handle(h)) return rc;
    if (int rc = check_buf(r, r_bytes, f64_planes(h, 1), "r")) return rc;
    if (int rc = check_buf(r_store, r_store_bytes, real_planes(h, 1), "r_store")) return rc;
    if (reinterpret_cast<uintptr_t>(r_store) % 16 != 0) return fail(ELBM_EINVAL, "r_store must be 16-byte aligned");
    if (int rc = set_device(h)) return rc;
    if (int rc = flush_pending(h)) return rc;
    HIP_OK(launch_source_field(h, r, r_store), "source field");
    h->r_mode = 2;
    h->r_field = r_store;
    return ELBM_OK;
}

int elbm_set_source_scale(elbm_lattice* h, double sc) {
    if (int rc = check_handle(h)) return rc;
    if (!std::isfinite(sc)) return fail(ELBM_EINVAL, "non-finite source scale");
    h->src_scale = sc;
    return ELBM_OK;
}

int elbm_clear_source(elbm_lattice* h) {
    if (int rc = check_handle(h)) return rc;
    if (int rc = set_device(h)) return rc;
    if (int rc = flush_pending(h)) return rc;
    h->r_mode = 0;
    h->r_field = nullptr;
    return ELBM_OK;
}

int elbm_set_dirichlet(elbm_lattice* h, double phi_lo, double phi_hi) {
    if (int r = check_handle(h)) return r;
    if (!std::isfinite(phi_lo) || !std::isfinite(phi_hi)) return fail(ELBM_EINVAL, "non-finite wall value");
    h->phi_lo = phi_lo;
    h->phi_hi = phi_hi;
    return ELBM_OK;
}

int elbm_init_equilibrium(elbm_lattice* h, const double* phi0, int64_t phi0_bytes, const double* j0,
                          int64_t j0_bytes) {
    if (int r = check_handle(h)) return r;
    if (int r = check_bound(h)) return r;
    if (int r = check_buf(phi0, phi0_bytes, f64_planes(h, 1), "phi0")) return r;
    if (int r = check_buf(j0, j0_bytes, f64_planes(h, 3), "j0", true)) return r;
    if (int r = set_device(h)) return r;
    HIP_OK(launch_init(h, phi0, j0, h->buf[h->cur]), "init");
    h->pending = false;
    h->initialized = true;
    h->time = 0;
    return ELBM_OK;
}

// One time step of the lattice's own run from src into dst (either may be a buffer other
// than the lattice's pair): the pending second source half-step of the previous step at its
// own amplitude plus the first half of this one, then the source and time bookkeeping.
static int advance(elbm_lattice* h, const void* src, void* dst, void* lam_rec, uint8_t* br_rec) {
    const double mult = (h->pending ? 0.5 * h->pending_scale : 0.0) + 0.5 * h->src_scale;
    HIP_OK(launch_step(h, src, dst, mult, lam_rec, br_rec), "step");
    h->pending = h->r_mode != 0;
    h->pending_scale = h->src_scale;
    h->time += 1;
    return ELBM_OK;
}

static int do_steps(elbm_lattice* h, int64_t n_steps, void* lam_rec, uint8_t* br_rec) {
    if (int r = check_handle(h)) return r;
    if (int r = check_bound(h)) return r;
    if (n_steps < 0) return fail(ELBM_EINVAL, "n_steps must be >= 0");
    if (!h->initialized) return fail(ELBM_ESTATE, "lattice not initialised");
    if (!h->t_set) return fail(ELBM_ESTATE, "diffusion tensor not set");
    if (int r = set_device(h)) return r;
    const int rb = real_bytes(h->cfg.precision);
    for (int64_t s = 0; s < n_steps; ++s) {
        void* lr = lam_rec ? static_cast<char*>(lam_rec) + s * h->n * rb : nullptr;
        uint8_t* br = br_rec ? br_rec + s * h->n : nullptr;
        if (int r = advance(h, h->buf[h->cur], h->buf[h->cur ^ 1], lr, br)) return r;
        h->cur ^= 1;
    }
    return ELBM_OK;
}

int elbm_step(elbm_lattice* h, int64_t n_steps) { return do_steps(h, n_steps, nullptr, nullptr); }

int elbm_step_record(elbm_lattice* h, int64_t n_steps, void* lambda_rec, int64_t lambda_bytes,
                     uint8_t* branch_rec, int64_t branch_bytes) {
    if (int r = check_handle(h)) return r;
    if (n_steps < 0) return fail(ELBM_EINVAL, "n_steps must be >= 0");
    if (int r = check_buf(lambda_rec, lambda_bytes, n_steps * real_planes(h, 1), "lambda_rec")) return r;
    if (int r = check_buf(branch_rec, branch_bytes, n_steps * h->n, "branch_rec")) return r;
    return do_steps(h, n_steps, lambda_rec, branch_rec);
}

int elbm_step_buffers(elbm_lattice* h, const void* src, int64_t src_bytes, int32_t pending, void* dst,
                      int64_t dst_bytes, void* lambda_rec, int64_t lambda_bytes, uint8_t* branch_rec,
                      int64_t branch_bytes) {
    if (int r = check_handle(h)) return r;
    if (!src || !dst || src == dst) return fail(ELBM_EINVAL, "need distinct source and destination buffers");
    if ((lambda_rec == nullptr) != (branch_rec == nullptr)) return fail(ELBM_EINVAL, "records come in pairs");
    if (int r = check_buf(src, src_bytes, pop_bytes(h), "src")) return r;
    if (int r = check_buf(dst, dst_bytes, pop_bytes(h), "dst")) return r;
    if (reinterpret_cast<uintptr_t>(src) % 16 != 0 || reinterpret_cast<uintptr_t>(dst) % 16 != 0)
        return fail(ELBM_EINVAL, "population buffers must be 16-byte aligned");
    if (int r = check_buf(lambda_rec, lambda_bytes, real_planes(h, 1), "lambda_rec", true)) return r;
    if (int r = check_buf(branch_rec, branch_bytes, h->n, "branch_rec", true)) return r;
    if (h->cfg.flags & (ELBM_FLAG_REST_FP32 | ELBM_FLAG_STOCHASTIC_ROUNDING))
        return fail(ELBM_EINVAL, "the adjoint entry points do not take rest-in-FP32 or stochastic-rounding storage");
    if (!h->t_set) return fail(ELBM_ESTATE, "diffusion tensor not set");
    if (int r = set_device(h)) return r;
    const double mult = ((pending && h->r_mode != 0) ? 1.0 : 0.5) * h->src_scale;
    HIP_OK(launch_step(h, src, dst, mult, lambda_rec, branch_rec), "step buffers");
    return ELBM_OK;
}

int elbm_read_moments(elbm_lattice* h, double* phi, int64_t phi_bytes, double* q3, int64_t q3_bytes) {
    if (int r = check_handle(h)) return r;
    if (int r = check_bound(h)) return r;
    if (int r = check_buf(phi, phi_bytes, f64_planes(h, 1), "phi", true)) return r;
    if (int r = check_buf(q3, q3_bytes, f64_planes(h, 3), "q3", true)) return r;
    if (!h->initialized) return fail(ELBM_ESTATE, "lattice not initialised");
    if (!h->t_set && q3) return fail(ELBM_ESTATE, "diffusion tensor not set");
    if (!phi && !q3) return ELBM_OK;
    if (int r = set_device(h)) return r;
    HIP_OK(launch_moments(h, phi, q3), "moments");
    return ELBM_OK;
}

int elbm_reduce(elbm_lattice* h, double* out4) {
    if (int r = check_handle(h)) return r;
    if (int r = check_bound(h)) return r;
    if (!out4) return fail(ELBM_EINVAL, "null output");
    if (!h->initialized) return fail(ELBM_ESTATE, "lattice not initialised");
    if (!h->t_set) return fail(ELBM_ESTATE, "diffusion tensor not set");
    if (int r = set_device(h)) return r;
    double* dout = h->d_part + 4 * h->part_blocks;
    HIP_OK(launch_reduce(h, dout, h->d_part), "reduce");
    HIP_OK(hipMemcpyAsync(out4, dout, 4 * sizeof(double), hipMemcpyDeviceToHost, h->stream), "reduce copy");
    HIP_OK(hipStreamSynchronize(h->stream), "reduce sync");
    return ELBM_OK;
}

int elbm_reduce_noalloc(elbm_lattice* h, double* out4, int64_t out4_bytes) {
    if (int r = check_handle(h)) return r;
    if (int r = check_bound(h)) return r;
    if (int r = check_buf(out4, out4_bytes, 4 * int64_t(sizeof(double)), "out4")) return r;
    if (!h->initialized) return fail(ELBM_ESTATE, "lattice not initialised");
    if (!h->t_set) return fail(ELBM_ESTATE, "diffusion tensor not set");
    if (h->part_blocks > kMaxPartBlocks)
        return fail(ELBM_ESHAPE, "the reduction needs more block partials than the static scratch holds (2048)");
    if (int r = set_device(h)) return r;
    double* part = static_cast<double*>(scratch_of(h->device));
    if (!part) return fail(ELBM_ESTATE, "static scratch not resolved on this device");
    HIP_OK(launch_reduce(h, out4, part), "reduce (static scratch)");
    return ELBM_OK;
}

int elbm_min_population(elbm_lattice* h, double* out) {
    if (int r = check_handle(h)) return r;
    if (int r = check_bound(h)) return r;
    if (!out) return fail(ELBM_EINVAL, "null output");
    if (!h->initialized) return fail(ELBM_ESTATE, "lattice not initialised");
    if (int r = set_device(h)) return r;
    double* dout = h->d_part + 4 * h->part_blocks + 4;  // past the four sums of elbm_reduce
    HIP_OK(launch_min_population(h, dout), "min population");
    HIP_OK(hipMemcpyAsync(out, dout, sizeof(double), hipMemcpyDeviceToHost, h->stream), "min population copy");
    HIP_OK(hipStreamSynchronize(h->stream), "min population sync");
    return ELBM_OK;
}

int elbm_stream_copy(elbm_lattice* h, const void* src, int64_t src_bytes, void* dst, int64_t dst_bytes) {
    if (int r = check_handle(h)) return r;
    if (!src || !dst) return fail(ELBM_EINVAL, "null buffer");
    const int64_t bytes = src_bytes;
    if (bytes <= 0 || bytes % 16 != 0) return fail(ELBM_EINVAL, "copy size must be a positive multiple of 16 bytes");
    if (dst_bytes < bytes) return fail(ELBM_ESHAPE, "dst smaller than src");
    const uintptr_t s = reinterpret_cast<uintptr_t>(src), d = reinterpret_cast<uintptr_t>(dst);
    if (s % 16 != 0 || d % 16 != 0) return fail(ELBM_EINVAL, "copy buffers must be 16-byte aligned");
    if (s < d + uintptr_t(bytes) && d < s + uintptr_t(bytes)) return fail(ELBM_EINVAL, "copy buffers overlap");
    if (int r = set_device(h)) return r;
    HIP_OK(launch_stream_copy(h, src, dst, size_t(bytes) / 16), "stream copy");
    return ELBM_OK;
}

int elbm_get_populations(elbm_lattice* h, double* f, int64_t f_bytes) {
    if (int r = check_handle(h)) return r;
    if (int r = check_bound(h)) return r;
    if (int r = check_buf(f, f_bytes, f64_planes(h, Q), "f")) return r;
    if (!h->initialized) return fail(ELBM_ESTATE, "lattice not initialised");
    if (int r = set_device(h)) return r;
    HIP_OK(launch_get_pops(h, f), "get populations");
    return ELBM_OK;
}

int elbm_set_populations(elbm_lattice* h, const double* f, int64_t f_bytes) {
    if (int r = check_handle(h)) return r;
    if (int r = check_bound(h)) return r;
    if (int r = check_buf(f, f_bytes, f64_planes(h, Q), "f")) return r;
    if (int r = set_device(h)) return r;
    HIP_OK(launch_set_pops(h, f, h->buf[h->cur]), "set populations");
    h->pending = false;
    h->initialized = true;
    return ELBM_OK;
}

int elbm_save_state(elbm_lattice* h, void* dst, int64_t dst_bytes, int64_t* step, int32_t* pending) {
    if (int r = check_handle(h)) return r;
    if (int r = check_bound(h)) return r;
    if (int r = check_buf(dst, dst_bytes, pop_bytes(h), "dst")) return r;
    if (int r = set_device(h)) return r;
    HIP_OK(hipMemcpyAsync(dst, h->buf[h->cur], size_t(elbm_population_bytes(h)),
                          hipMemcpyDeviceToDevice, h->stream), "save state");
    if (step) *step = h->time;
    if (pending) *pending = h->pending ? 1 : 0;
    return ELBM_OK;
}

int elbm_load_state(elbm_lattice* h, const void* src, int64_t src_bytes, int64_t step, int32_t pending) {
    if (int r = check_handle(h)) return r;
    if (int r = check_bound(h)) return r;
    if (int r = check_buf(src, src_bytes, pop_bytes(h), "src")) return r;
    if (int r = set_device(h)) return r;
    HIP_OK(hipMemcpyAsync(h->buf[h->cur], src, size_t(elbm_population_bytes(h)),
                          hipMemcpyDeviceToDevice, h->stream), "load state");
    h->time = step;
    h->pending = pending != 0 && h->r_mode != 0;
    h->pending_scale = h->src_scale;
    h->initialized = true;
    return ELBM_OK;
}

int elbm_adjoint_step(elbm_lattice* h, const void* state, int64_t state_bytes, int32_t pending,
                      const void* lambda_rec, int64_t lambda_bytes, const uint8_t* branch_rec,
                      int64_t branch_bytes, const void* adj_in, int64_t adj_in_bytes, void* adj_out,
                      int64_t adj_out_bytes, void* t_grad, int64_t t_grad_bytes) {
    if (int r = check_handle(h)) return r;
    if (int r = check_buf(state, state_bytes, pop_bytes(h), "state")) return r;
    if (int r = check_buf(lambda_rec, lambda_bytes, real_planes(h, 1), "lambda_rec")) return r;
    if (int r = check_buf(branch_rec, branch_bytes, h->n, "branch_rec")) return r;
    if (int r = check_buf(adj_in, adj_in_bytes, real_planes(h, Q), "adj_in")) return r;
    if (int r = check_buf(adj_out, adj_out_bytes, real_planes(h, Q), "adj_out")) return r;
    if (int r = check_buf(t_grad, t_grad_bytes, real_planes(h, 6), "t_grad")) return r;
    if (adj_in == adj_out) return fail(ELBM_EINVAL, "adj_in and adj_out must not alias");
    if (reinterpret_cast<uintptr_t>(t_grad) % 16 != 0) return fail(ELBM_EINVAL, "t_grad must be 16-byte aligned");
    if (int r = adjoint_ready(h)) return r;
    if (int r = set_device(h)) return r;
    HIP_OK(launch_adjoint(h, state, replay_mult(h, pending != 0), lambda_rec, branch_rec, adj_in, adj_out,
                          t_grad),
           "adjoint step");
    return ELBM_OK;
}

int64_t elbm_gradient_workspace_bytes(const elbm_lattice* h, int64_t steps, int64_t ckpt) {
    if (!h) return fail(ELBM_EINVAL, "null lattice handle");
    if (steps < 1 || ckpt < 1) return fail(ELBM_EINVAL, "steps and ckpt must be >= 1");
    return int64_t(sweep_layout(h, steps, ckpt).total);
}

int elbm_forward_record(elbm_lattice* h, int64_t steps, int64_t ckpt, void* workspace,
                        int64_t workspace_bytes) {
    if (int r = check_handle(h)) return r;
    if (int r = check_bound(h)) return r;
    if (steps < 1 || ckpt < 1) return fail(ELBM_EINVAL, "steps and ckpt must be >= 1");
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(ELBM_EINVAL, "workspace must be a 256-byte aligned device buffer");
    if (int r = check_buf(workspace, workspace_bytes, int64_t(sweep_layout(h, steps, ckpt).total), "workspace"))
        return r;
    if (!h->initialized) return fail(ELBM_ESTATE, "lattice not initialised");
    if (int r = adjoint_ready(h)) return r;
    if (int r = set_device(h)) return r;
    const SweepLayout L = sweep_layout(h, steps, ckpt);
    char* w = static_cast<char*>(workspace);
    const size_t n = size_t(h->n), rb = size_t(real_bytes(h->cfg.precision));
    h->rec_ws = nullptr;  // invalid until the run completes
    h->rec_last_kept = false;
    h->rec_pending0 = h->pending;
    for (int64_t s = 0; s < steps; s += ckpt) {
        const int64_t m = (steps - s < ckpt) ? steps - s : ckpt;
        void* lam = w + L.lam + size_t(s) * n * rb;
        uint8_t* br = reinterpret_cast<uint8_t*>(w + L.br) + size_t(s) * n;
        HIP_OK(hipMemcpyAsync(w + L.ck + size_t(s / ckpt) * L.pop, h->buf[h->cur],
                              size_t(elbm_population_bytes(h)), hipMemcpyDeviceToDevice, h->stream),
               "checkpoint");
        if (s + m < steps) {
            if (int r = do_steps(h, m, lam, br)) return r;
            continue;
        }
        // last segment: its states 1 .. m - 1 go straight into the sweep's recompute buffers,
        // so the reverse sweep starts without recomputing them; the last step lands in the
        // lattice's own buffer
        if (int r = check_bound(h)) return r;
        for (int64_t j = 0; j < m; ++j) {
            const void* src = j == 0 ? h->buf[h->cur] : w + L.seg + size_t(j - 1) * L.pop;
            void* dst = j + 1 < m ? w + L.seg + size_t(j) * L.pop : h->buf[h->cur ^ 1];
            if (int r = advance(h, src, dst, static_cast<char*>(lam) + size_t(j) * n * rb, br + size_t(j) * n))
                return r;
        }
        h->cur ^= 1;
    }
    h->rec_steps = steps;
    h->rec_ckpt = ckpt;
    h->rec_ws = workspace;
    h->rec_last_kept = true;
    return ELBM_OK;
}

int elbm_gradient(elbm_lattice* h, int64_t steps, int64_t ckpt, void* workspace, int64_t workspace_bytes,
                  const double* dphi_n, int64_t dphi_n_bytes, void* t_grad, int64_t t_grad_bytes,
                  double* dphi0, int64_t dphi0_bytes, double* dj0, int64_t dj0_bytes) {
    if (int r = check_handle(h)) return r;
    if (steps < 1 || ckpt < 1) return fail(ELBM_EINVAL, "steps and ckpt must be >= 1");
    if (int r = check_buf(workspace, workspace_bytes, int64_t(sweep_layout(h, steps, ckpt).total), "workspace"))
        return r;
    if (int r = check_buf(dphi_n, dphi_n_bytes, f64_planes(h, 1), "dphi_n")) return r;
    if (int r = check_buf(t_grad, t_grad_bytes, real_planes(h, 6), "t_grad")) return r;
    if (int r = check_buf(dphi0, dphi0_bytes, f64_planes(h, 1), "dphi0", true)) return r;
    if (int r = check_buf(dj0, dj0_bytes, f64_planes(h, 3), "dj0", true)) return r;
    if (reinterpret_cast<uintptr_t>(t_grad) % 16 != 0) return fail(ELBM_EINVAL, "t_grad must be 16-byte aligned");
    if (h->rec_ws != workspace || h->rec_steps != steps || h->rec_ckpt != ckpt)
        return fail(ELBM_ESTATE, "no elbm_forward_record with these steps, ckpt and workspace");
    if (int r = adjoint_ready(h)) return r;
    if (int r = set_device(h)) return r;
    const SweepLayout L = sweep_layout(h, steps, ckpt);
    char* w = static_cast<char*>(workspace);
    const size_t n = size_t(h->n), rb = size_t(real_bytes(h->cfg.precision));
    const bool has_src = h->r_mode != 0;
    void* cur = w + L.adj;
    void* nxt = w + L.adj + L.adj_bytes;
    HIP_OK(launch_fill_adjoint(h, dphi_n, cur), "adjoint of the readout");
    for (int64_t seg = L.nck - 1; seg >= 0; --seg) {
        const int64_t s0 = seg * ckpt;
        const int64_t m = (steps - s0 < ckpt) ? steps - s0 : ckpt;
        // state j of the segment: the checkpoint for j = 0, recomputed buffer j - 1 after it
        auto state = [&](int64_t j) -> char* {
            return j == 0 ? w + L.ck + size_t(seg) * L.pop : w + L.seg + size_t(j - 1) * L.pop;
        };
        auto pend = [&](int64_t j) { return (seg == 0 && j == 0) ? h->rec_pending0 : has_src; };
        // the newest segment's states are still in the buffers from the forward run, unless
        // an earlier sweep has overwritten them
        const bool kept = seg == L.nck - 1 && h->rec_last_kept;
        if (seg == L.nck - 1) h->rec_last_kept = false;  // older segments reuse the buffers
        for (int64_t j = 0; !kept && j + 1 < m; ++j)
            HIP_OK(launch_step(h, state(j), state(j + 1), replay_mult(h, pend(j)), nullptr, nullptr), "recompute");
        for (int64_t j = m - 1; j >= 0; --j) {
            const size_t s = size_t(s0 + j);
            HIP_OK(launch_adjoint(h, state(j), replay_mult(h, pend(j)), w + L.lam + s * n * rb,
                                  reinterpret_cast<uint8_t*>(w + L.br) + s * n, cur, nxt, t_grad),
                   "adjoint step");
            void* t = cur;
            cur = nxt;
            nxt = t;
        }
    }
    if (dphi0) HIP_OK(launch_init_gradient(h, cur, dphi0, dj0), "initial gradient");
    return ELBM_OK;
}

int elbm_tensor_gradient(elbm_lattice* h, const double* d6, int64_t d6_bytes, int32_t is_log,
                         const void* t_grad, int64_t t_grad_bytes, double* out6, int64_t out6_bytes) {
    if (int r = check_handle(h)) return r;
    if (int r = check_buf(d6, d6_bytes, f64_planes(h, 6), "d6")) return r;
    if (int r = check_buf(t_grad, t_grad_bytes, real_planes(h, 6), "t_grad")) return r;
    if (int r = check_buf(out6, out6_bytes, f64_planes(h, 6), "out6")) return r;
    if (int r = set_device(h)) return r;
    HIP_OK(launch_tensor_gradient(h, d6, is_log ? 1 : 0, t_grad, out6), "tensor gradient");
    return ELBM_OK;
}

int elbm_initial_gradient(elbm_lattice* h, const void* adj0, int64_t adj0_bytes, double* dphi0,
                          int64_t dphi0_bytes, double* dj0, int64_t dj0_bytes) {
    if (int r = check_handle(h)) return r;
    if (int r = check_buf(adj0, adj0_bytes, real_planes(h, Q), "adj0")) return r;
    if (int r = check_buf(dphi0, dphi0_bytes, f64_planes(h, 1), "dphi0")) return r;
    if (int r = check_buf(dj0, dj0_bytes, f64_planes(h, 3), "dj0", true)) return r;
    if (int r = set_device(h)) return r;
    HIP_OK(launch_init_gradient(h, adj0, dphi0, dj0), "initial gradient");
    return ELBM_OK;
}

int elbm_get_counters(elbm_lattice* h, elbm_counters* out) {
    if (int r = check_handle(h)) return r;
    if (!out) return fail(ELBM_EINVAL, "null output");
    if (int r = set_device(h)) return r;
    std::vector<unsigned long long> w(kCntWords);
    HIP_OK(hipMemcpyAsync(w.data(), h->d_cnt, kCntWords * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                          h->stream), "counters");
    HIP_OK(hipStreamSynchronize(h->stream), "counters sync");
    unsigned long long c[kNumCounters] = {0, 0, 0, 0};
    for (int m = 0; m < kNumCounters; ++m)
        for (unsigned slot = 0; slot < unsigned(kCntSlots); ++slot) c[m] += w[cnt_index(m, slot)];
    out->fallback_nodes = c[0];
    out->flagged_nodes = c[1];
    out->nonfinite = c[2];
    out->guard_nodes = c[3];
    return ELBM_OK;
}

int elbm_reset_counters(elbm_lattice* h) {
    if (int r = check_handle(h)) return r;
    if (int r = set_device(h)) return r;
    HIP_OK(hipMemsetAsync(h->d_cnt, 0, kCntWords * sizeof(unsigned long long), h->stream), "reset counters");
    return ELBM_OK;
}

int64_t elbm_time(const elbm_lattice* h) { return h ? h->time : -1; }

}  // extern "C"
