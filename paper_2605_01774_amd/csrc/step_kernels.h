// Fused collide-and-stream step kernel and its adjoint (reverse) step kernel (D3Q19 or D3Q27).
// Included by one translation unit per storage form (step_f64.hip, step_f32.hip,
// step_bf16.hip, step_fp16.hip), which instantiate the host launchers below.
//
// Forward (one launch per time step): each thread owns one node x. It reads the Q
// pre-collision populations of x (coalesced: x is fastest in every run of a row), adds the
// pending source half-steps, collides in registers (node.h), and pushes post_i to
// x + c_i in the other buffer (periodic in y and z; periodic or anti-bounce-back on the x
// faces). Every stored value is read once and written once per step, so the kernel moves
// exactly 2 Q stored values per node plus the per-node fields it is given.
//
// Adjoint (one launch per reverse step): each thread gathers dL/dg_{t+1} from x + c_i (the
// transpose of the push), recomputes the node's collision from the saved state, applies
// the vector-Jacobian product and writes dL/dg_t at x; dL/dT is accumulated per node.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "args.h"

namespace elbm {

// Storage rounding of the values a node is about to store (16-bit forms with
// ELBM_FLAG_REST_FP32 or ELBM_FLAG_STOCHASTIC_ROUNDING: the RS instantiations of the step
// kernels; otherwise the stores round to nearest even themselves). Each 16-bit value is
// rounded here, so the stores convert exactly. With the FP32 rest population the rest value
// takes up the rounding of the 18 others, which keeps the node's stored mass equal to the
// computed one: the rest value becomes the node's mass after the collision, which the
// collision conserves (dphi, source included; at a Dirichlet plane plus what the reflection
// there changed), minus the rounded moving populations. Random bits: RoundingBits seeded
// with the node index mixed with a hash of the time step. The rounded 16-bit values are left
// in storage units (FP16: value / scale, exact for the power-of-two scale), which the stores
// of these kernels take unscaled; the FP32 rest value is in physical units. Their sum times
// the scale equals the sum of the scaled values bit for bit, so the results are the same as
// with physical values, two multiplies per value fewer in FP16.
// SU: the node's values are already in storage units (the FP16 step in storage units).
template <class ST, bool SR, bool REST, bool SU, class Real>
__device__ inline void round_node(Real (&post)[Q], const StepArgs<Real>& a, uint32_t k, Real mass) {
    const Real scale = SU ? Real(1) : a.scale, inv_scale = SU ? Real(1) : a.inv_scale;
    RoundingBits rb(k ^ a.tmix);
    Real res = Real(0);  // REST: sum of the rounded moving populations, storage units
    if constexpr (SR) {
        // one 32-bit word per opposite pair (P, P + 1)
#pragma unroll
        for (int P = 1; P < Q; P += 2) {
            Real q0, q1;
            quantize16_sr_pair<ST, true>(post[P], post[P + 1], rb.next(), scale, inv_scale, q0, q1);
            if constexpr (REST) {
                res += q0;
                res += q1;
            }
            post[P] = q0;
            post[P + 1] = q1;
        }
    } else {
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const Real q = quantize16<ST, true>(post[i], 0u, false, scale, inv_scale);
            if constexpr (REST) res += q;
            post[i] = q;
        }
    }
    if constexpr (REST)
        post[0] = mass - ((std::is_same<ST, bf16s>::value || SU) ? res : res * scale);
    else
        post[0] = quantize16<ST, true>(post[0], SR ? rb.next() : 0u, SR, scale, inv_scale);
}

// mass: the node's mass after the collision and the wall reflection (used with the FP32 rest)
template <class ST, bool SU, class Real>
__device__ inline void store_rounding(Real (&post)[Q], const StepArgs<Real>& a, uint32_t k, Real mass) {
    if constexpr (sizeof(ST) == 2) {
        // the two options are uniform over the launch: one branch per node, none per value
        if (a.sround) {
            if (a.rest32) round_node<ST, true, true, SU>(post, a, k, mass);
            else round_node<ST, true, false, SU>(post, a, k, mass);
        } else if (a.rest32) {
            round_node<ST, false, true, SU>(post, a, k, mass);
        }
    }
}

// Halfway anti-bounce-back, in place: at a Dirichlet plane the population leaving the
// domain becomes the opposite population of the same node, g_opp = -post_i + 2 W_i phi_w
// (deviation form: minus W_i phi_ref); post[i] then holds the value for direction opp(i).
// mass takes up the change of the node's mass.
template <class Real>
__device__ inline void reflect_at_walls(Real (&post)[Q], bool lo, bool hi, Real phi_lo, Real phi_hi,
                                        Real phi_ref, Real& mass) {
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        if (lo && cx(i) == -1) {
            const Real g = -post[i] + Real(2.0 * weight(i)) * (phi_lo - phi_ref);
            mass += g - post[i];
            post[i] = g;
        }
        if (hi && cx(i) == 1) {
            const Real g = -post[i] + Real(2.0 * weight(i)) * (phi_hi - phi_ref);
            mass += g - post[i];
            post[i] = g;
        }
    }
}

// FP16 storage runs the step in storage units (value / scale, the scale a power of two): the
// 16-bit populations are loaded and stored unscaled, the FP32 rest population (RS) is
// scaled on its way in and out, and the physical constants (phi_ref, eps, the source, the
// wall values) are scaled instead. Every operation of the update is homogeneous of degree
// one in these (lambda and alpha are ratios of exactly scaled sums, the storage rounding
// sees the same values), so the stored results are bitwise those of the step in physical
// units, with two multiplies per population fewer. The exact-root variant, whose logarithms
// are of the populations themselves, keeps physical units.
template <class ST, bool RS, bool ROOT>
constexpr bool storage_units() {
    return std::is_same<ST, _Float16>::value && !ROOT;
}

template <class ST, int UM, bool ROOT, bool ABB, bool RS>
__global__ __launch_bounds__(512) void k_step(const StepArgs<typename Store<ST>::Real> a) {
    using Real = typename Store<ST>::Real;
    constexpr bool SU = storage_units<ST, RS, ROOT>();
    const Real su = SU ? a.inv_scale : Real(1);  // physical value -> storage units
    const int rest32 = RS ? a.rest32 : 0;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= a.nx || y >= a.ny) return;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int nxy = nx * ny;
    const int k = z * nxy + y * nx + x;
    const int r = z * ny + y;  // row
    const ST* src = static_cast<const ST*>(a.src);
    ST* dst = static_cast<ST*>(a.dst);

    Real d[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i] = pop_load<ST>(src, i, r, x, nx, rest32, SU ? Real(1) : a.scale);
    if (SU && rest32) d[0] *= a.inv_scale;  // the FP32 rest value is stored in physical units

    NodeCoef<Real> c;
    node_coef<Real, UM>(a, k, c);
    if (a.has_src) {
        const Real R = ((a.rfield ? a.rfield[k] : a.R) * a.src_mult) * su;
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] += R * Real(weight(i)) * (Real(1) + c.ex[i]);
    }

    Real post[Q];
    NodeOut<Real> o;
    collide<Real, UM, ROOT, sizeof(ST) == 4, sizeof(ST) != 2>(d, c, a.phi_ref * su, a.eps * su, a.tau2, a.root_rho,
                                                              post, o);

    if (a.lam_rec) {
        a.lam_rec[k] = o.lam;
        a.br_rec[k] = uint8_t(o.branch);
    }
    if (a.counters) {
        const unsigned slot = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
        if (o.branch != 255) atomicAdd(a.counters + cnt_index(0, slot), 1ull);
        if (o.flagged) atomicAdd(a.counters + cnt_index(1, slot), 1ull);
        if (!isfinite(o.dphi)) atomicAdd(a.counters + cnt_index(2, slot), 1ull);
        if (o.guard) atomicAdd(a.counters + cnt_index(3, slot), 1ull);
    }

    const bool lo = ABB && x == 0, hi = ABB && x == nx - 1;
    // RS: store_rounding leaves the 16-bit values in storage units, stored unscaled
    const Real st_inv = (RS || SU) ? Real(1) : a.inv_scale;
    Real mass = o.dphi;
    if (ABB) reflect_at_walls(post, lo, hi, a.phi_lo * su, a.phi_hi * su, a.phi_ref * su, mass);
    if constexpr (RS) store_rounding<ST, SU>(post, a, uint32_t(k), mass);
    if (SU && rest32) post[0] *= a.scale;

    // push streaming
    const int xm = (x == 0) ? nx - 1 : x - 1, xp = (x == nx - 1) ? 0 : x + 1;
    const int ym = (y == 0) ? ny - 1 : y - 1, yp = (y == ny - 1) ? 0 : y + 1;
    const int zm = (z == 0) ? nz - 1 : z - 1, zp = (z == nz - 1) ? 0 : z + 1;
    const int ox[3] = {xm, x, xp};
    const int ry[3] = {ym, y, yp};
    const int rz[3] = {zm * ny, z * ny, zp * ny};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if ((cx(i) == 1 && hi) || (cx(i) == -1 && lo)) {
            // reflected at a Dirichlet plane: stays at this node as the opposite population
            pop_put<ST>(dst, opp(i), r, x, nx, post[i], rest32, st_inv);
        } else {
            pop_put<ST>(dst, i, rz[cz(i) + 1] + ry[cy(i) + 1], ox[cx(i) + 1], nx, post[i], rest32, st_inv);
        }
    }
}

// ------------------------------------------------------------------------------------------
// Row-vector variant for rows of nx = 64 V W nodes (W <= 8): one block holds whole rows,
// lane l of wavefront w owns the V consecutive nodes x = V (64 w + l) .. + V - 1, so every
// population run of the row is read and written with one V-wide access per lane. The +-1
// x-shift of the directions with c_x != 0 is a rotation of the row by one node: one element
// crosses to the neighbouring lane, which a single DPP wavefront rotate provides, and
// values crossing between the wavefronts of a row go through LDS.
//
// Periodic rows close the rotation (x = nx - 1 <-> x = 0). With Dirichlet x faces (ABB)
// the two wrapped elements are not stored; instead each wall node writes its reflected
// populations at its own position, exactly as the one-node-per-thread kernel does.
// ------------------------------------------------------------------------------------------
//
// Every population access of this kernel is a nontemporal load or store (the buffers
// are streamed once per step and are far larger than the caches): on MI355X this measured
// 3-5 % faster than plain accesses at 256^3 (FP32 423 vs 446 us, BF16 219 vs 227 us, FP64
// 874 vs 908 us per step), while nontemporal stores slowed the one-node-per-thread kernel,
// whose x-shifted stores write lines partially, by 12-15 %.
template <class ST, int V>
struct VecIO {
    using Real = typename Store<ST>::Real;
    static constexpr int BYTES = int(sizeof(ST)) * V;
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    using Raw = typename std::conditional<BYTES == 16, u32x4,
                typename std::conditional<BYTES == 8, u32x2,
                typename std::conditional<BYTES == 4, uint32_t, uint16_t>::type>::type>::type;
    static constexpr int WORDS = BYTES >= 4 ? BYTES / 4 : 1;

    // 16-bit value <-> arithmetic type
    __device__ static inline Real from16(uint32_t bits, Real scale) {
        if constexpr (std::is_same<ST, bf16s>::value) {
            return __uint_as_float(bits << 16);
        } else {
            return float(__builtin_bit_cast(_Float16, uint16_t(bits))) * scale;
        }
    }
    __device__ static inline uint32_t to16(Real v, Real inv_scale) {
        if constexpr (std::is_same<ST, bf16s>::value) {
            return __builtin_bit_cast(uint16_t, static_cast<__bf16>(v));
        } else {
            return __builtin_bit_cast(uint16_t, _Float16(v * inv_scale));
        }
    }
    // two values into one 32-bit word (v0 in the low half): one packed round-to-nearest-even
    // conversion (v_cvt_pk_bf16_f32 / v_cvt_pk_f16_f32), bitwise the same as two to16
    __device__ static inline uint32_t pack16(Real v0, Real v1, Real inv_scale) {
        typedef float f2 __attribute__((ext_vector_type(2)));
        if constexpr (std::is_same<ST, bf16s>::value) {
            return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2{v0, v1}, bf16x2));
        } else {
            return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2{v0 * inv_scale, v1 * inv_scale}, f16x2));
        }
    }

    __device__ static inline void load(const ST* p, Real (&out)[V], Real scale) {
        const Raw raw = __builtin_nontemporal_load(reinterpret_cast<const Raw*>(p));
        if constexpr (BYTES == 2) {
            out[0] = from16(uint32_t(raw), scale);
        } else {
            uint32_t w[WORDS];
            __builtin_memcpy(w, &raw, sizeof(w));
            if constexpr (sizeof(ST) == 8) {
#pragma unroll
                for (int e = 0; e < V; ++e) out[e] = __hiloint2double(int(w[2 * e + 1]), int(w[2 * e]));
            } else if constexpr (sizeof(ST) == 4) {
#pragma unroll
                for (int e = 0; e < V; ++e) out[e] = __uint_as_float(w[e]);
            } else {
#pragma unroll
                for (int e = 0; e < V; ++e) out[e] = from16((e & 1) ? (w[e >> 1] >> 16) : (w[e >> 1] & 0xFFFFu), scale);
            }
        }
    }

    __device__ static inline void store(ST* p, const Real (&in)[V], Real inv_scale) {
        Raw raw;
        if constexpr (BYTES == 2) {
            raw = uint16_t(to16(in[0], inv_scale));
        } else {
            uint32_t w[WORDS];
            if constexpr (sizeof(ST) == 8) {
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    w[2 * e] = uint32_t(__double2loint(in[e]));
                    w[2 * e + 1] = uint32_t(__double2hiint(in[e]));
                }
            } else if constexpr (sizeof(ST) == 4) {
#pragma unroll
                for (int e = 0; e < V; ++e) w[e] = __float_as_uint(in[e]);
            } else {
#pragma unroll
                for (int e = 0; e < V; e += 2) w[e >> 1] = pack16(in[e], in[e + 1], inv_scale);
            }
            __builtin_memcpy(&raw, w, sizeof(w));
        }
        __builtin_nontemporal_store(raw, reinterpret_cast<Raw*>(p));
    }
};

// Rotate one value across the wavefront: lane l receives the value of lane l - 1 (DIR = +1)
// or lane l + 1 (DIR = -1), modulo 64.
template <int DIR>
__device__ inline float wave_rotate(float v) {
    constexpr int ctrl = DIR > 0 ? 0x13C : 0x134;  // DPP wave_ror:1 / wave_rol:1
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), ctrl, 0xF, 0xF, false));
}
template <int DIR>
__device__ inline double wave_rotate(double v) {
    constexpr int ctrl = DIR > 0 ? 0x13C : 0x134;
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), ctrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// N consecutive values of the arithmetic type from p, whose byte address is a multiple of
// the largest of 16, 8, 4 that divides N sizeof(Real): in loads of that many bytes.
template <class Real, int N>
__device__ inline void load_span(const Real* p, Real (&out)[N]) {
    constexpr int BYTES = N * int(sizeof(Real));
    constexpr int CH = BYTES % 16 == 0 ? 16 : (BYTES % 8 == 0 ? 8 : 4);
    constexpr int PER = CH / int(sizeof(Real));
    static_assert(PER >= 1 && N % PER == 0, "span must split into chunks");
#pragma unroll
    for (int j = 0; j < N / PER; ++j) {
        Real t[PER];
        VecIO<Real, PER>::load(p + j * PER, t, Real(1));
#pragma unroll
        for (int e = 0; e < PER; ++e) out[j * PER + e] = t[e];
    }
}

// Block order of the row-vector kernel. The dispatcher deals consecutive workgroups (x
// fastest, then y, then z) to the eight XCDs in turn, and each XCD has its own L2 and
// address-translation caches. In the natural order the XCDs take every eighth row of the
// same planes, so each of them touches the whole of the few planes being read and written
// (tens of MB at 512^3). With the remap, when the grid has a multiple of 8 blocks along y
// and z, block (by, bz) runs on XCD x = by mod 8 and is given the row block
//   ty = (gy / 8) (bz mod 8) + by / 8,   tz = (nz / 8) x + bz / 8,
// so that XCD x sweeps the contiguous slab of planes x nz/8 .. (x + 1) nz/8 - 1, row block
// by row block, plane by plane. The map is a bijection of the grid (mixed radix 8, gy/8, 8,
// nz/8) and uses shifts, masks and one product only.
__device__ inline void xcd_block(unsigned by, unsigned bz, unsigned gy, unsigned gz, bool remap, int& ty, int& tz) {
    if (!remap) {
        ty = int(by);
        tz = int(bz);
        return;
    }
    ty = int((gy >> 3) * (bz & 7u) + (by >> 3));
    tz = int((gz >> 3) * (by & 7u) + (bz >> 3));
}

template <class ST, int UM, int V, int W, bool ABB, bool RS>
__global__ __launch_bounds__(W > 4 ? 64 * W : 256) void k_step_vec(const StepArgs<typename Store<ST>::Real> a) {
    using Real = typename Store<ST>::Real;
    using IO = VecIO<ST, V>;
    constexpr bool SU = storage_units<ST, RS, false>();
    const Real su = SU ? a.inv_scale : Real(1);  // physical value -> storage units
    constexpr int ROWS = (W == 3 || W > 4) ? 1 : 4 / W;  // rows per block (blockDim.y)
    // values crossing between the wavefronts of a row: [row][wave][direction]
    __shared__ Real xfer[ROWS][W > 1 ? W : 1][Q];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;  // wavefront within the row
    // A wavefront lies in one row (blockDim.x is a multiple of 64), so threadIdx.y is uniform
    // across its lanes: read through readfirstlane, the row and every row offset below stay
    // in scalar registers, and each access is a scalar row base plus the lane's column.
    const int ty = ROWS == 1 ? 0 : __builtin_amdgcn_readfirstlane(int(threadIdx.y));
    int by, z;
    // the grid is ((ny + ROWS - 1) / ROWS, nz) blocks in y and z (from the arguments, which
    // the wave has already loaded, rather than from the dispatch packet)
    xcd_block(blockIdx.y, blockIdx.z, unsigned((a.ny + ROWS - 1) / ROWS), unsigned(a.nz), a.xcd_remap != 0, by, z);
    const int y = by * ROWS + ty;
    const bool active = y < a.ny;  // uniform per wavefront
    if (W == 1 && !active) return;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int xo = (w * 64 + lane) * V;
    const int r = z * ny + (active ? y : 0);  // row
    const long long kr = (long long)r * nx;   // node index of the row's x = 0
    // FP32 rest population of the 16-bit forms (ELBM_FLAG_REST_FP32)
    const int rest32 = (RS && sizeof(ST) == 2) ? a.rest32 : 0;
    const size_t re = row_elems(nx, rest32);
    const ST* src = static_cast<const ST*>(a.src);
    ST* dst = static_cast<ST*>(a.dst);
    const ST* srow = src + size_t(r) * re;
    // the per-node fields and records, moved to this row: node x of the row is entry xo + e
    StepArgs<Real> ar = a;
    if (ar.tfield && !ar.phase) ar.tfield += 6 * kr;
    if (ar.phase) ar.phase += kr;
    if (ar.ufield) ar.ufield += kr;
    if (ar.rfield) ar.rfield += kr;
    if (ar.lam_rec) ar.lam_rec += kr;
    if (ar.br_rec) ar.br_rec += kr;
    // wall lanes of a Dirichlet row: the node at x = 0 and the node at x = nx - 1
    const bool lo_wall = ABB && w == 0 && lane == 0;
    const bool hi_wall = ABB && w == W - 1 && lane == 63;

    // Per-node fields of the lane's V nodes, issued before the populations (FP64 and 16-bit
    // storage, up to two nodes per lane): loaded node by node after the populations and the
    // collision of the node before, each field cost the wave another memory round trip (FP64
    // field workload 512^3: 10.1-10.5 ms per step before, 8.7-9.0 ms with the early loads,
    // same boxes). The tensor is issued here too in the 16-bit forms when its rows come from a
    // material table (porous 384^3: 1-3 % faster) or with a velocity field (field workload
    // 512^3: 2-6 %); a per-node tensor without a velocity field is faster loaded at its use
    // (porous 384^3 with a tensor field: 5 % slower early). In FP64 its 6 V values would push
    // the two-node kernel past 256 VGPRs (one wave per SIMD), so there each node's tensor is
    // loaded just before its collision. At four nodes per lane (16-bit forms without a
    // velocity field) the early values cost 16-24 VGPRs, one wave per SIMD; with FP32 storage
    // (one node per lane, four waves per SIMD) they made the field workload 3-4 % slower.
    // There every field is loaded where it is used.
    constexpr bool PRE = V <= 2 && sizeof(ST) != 4;
    constexpr bool PRE_T = PRE && sizeof(Real) == 4;
    // A table of two materials (the two-phase media of Sec. 4.2.2) is read whole, at the same
    // address in every lane, and each node selects its row by its material index: no
    // per-node gather of the row, and no second memory round trip after the index. Porous
    // 384^3 (Dirichlet planes, u = 0), same box: BF16 2 % and BF16 + FP32 rest + SR 1.1 %
    // faster; FP32 storage 2 % (one node per lane) and 3 % (two) slower and FP64 unchanged.
    // So only the 16-bit wall kernels at u = 0 carry it: in the others the extra code cost
    // 0.2-1.2 % without a table (256^3 decay, 256^3 plume, 512^3 field workload).
    constexpr bool TWO = sizeof(ST) == 2 && UM == 0 && ABB;
    const bool two = TWO && ar.phase && a.phase_max == 1;  // uniform
    const bool t_early = PRE_T && active && ar.tfield && !two && (ar.phase || UM == 2);  // uniform
    Real tt[2][6];
    bool ph[V];
    if (two && active) {
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            tt[0][m] = ar.tfield[m];
            tt[1][m] = ar.tfield[6 + m];
        }
#pragma unroll
        for (int e = 0; e < V; ++e) ph[e] = ar.phase[xo + e] != 0;
    }
    Real uf[V][3], rf[V], tf[V][6];
#pragma unroll
    for (int e = 0; e < V; ++e) uf[e][0] = uf[e][1] = uf[e][2] = Real(0);
    if (PRE && active) {
        if (t_early) {
            if (!ar.phase) {
                Real t[6 * V];
                load_span(ar.tfield + 6 * xo, t);
#pragma unroll
                for (int e = 0; e < V; ++e)
#pragma unroll
                    for (int m = 0; m < 6; ++m) tf[e][m] = t[6 * e + m];
            } else {
#pragma unroll
                for (int e = 0; e < V; ++e) load_t6(ar.tfield, tensor_row(ar, xo + e), tf[e]);
            }
        }
        if constexpr (UM == 2) {
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                Real t[V];
                VecIO<Real, V>::load(ar.ufield + m * a.n + xo, t, Real(1));
#pragma unroll
                for (int e = 0; e < V; ++e) uf[e][m] = t[e];
            }
        }
        if (ar.rfield) {
            VecIO<Real, V>::load(ar.rfield + xo, rf, Real(1));
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) rf[e] = a.R;
        }
    }
    Real post[V][Q];
    if (active) {
        Real d[V][Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            Real t[V];
            bool done = false;
            if constexpr (sizeof(ST) == 2) {
                if (i == 0 && rest32) {
                    VecIO<float, V>::load(reinterpret_cast<const float*>(srow) + xo, t, 1.0f);
                    if constexpr (SU) {
#pragma unroll
                        for (int e = 0; e < V; ++e) t[e] *= a.inv_scale;
                    }
                    done = true;
                }
            }
            if (!done) IO::load(srow + run_offset(i, nx, rest32) + xo, t, SU ? Real(1) : a.scale);
#pragma unroll
            for (int e = 0; e < V; ++e) d[e][i] = t[e];
        }
#pragma unroll
        for (int e = 0; e < V; ++e) {
            NodeCoef<Real> c;
            if (two) {
                if constexpr (PRE)
                    coef_velocity<Real, UM>(a, uf[e][0], uf[e][1], uf[e][2], c);
                else
                    coef_velocity<Real, UM>(a, Real(0), Real(0), Real(0), c);
#pragma unroll
                for (int m = 0; m < 6; ++m) c.T[m] = ph[e] ? tt[1][m] : tt[0][m];
            } else if constexpr (PRE) {
                coef_velocity<Real, UM>(a, uf[e][0], uf[e][1], uf[e][2], c);
                if (t_early) {
#pragma unroll
                    for (int m = 0; m < 6; ++m) c.T[m] = tf[e][m];
                } else if (ar.tfield) {
                    load_t6(ar.tfield, tensor_row(ar, xo + e), c.T);
                } else {
#pragma unroll
                    for (int m = 0; m < 6; ++m) c.T[m] = a.T[m];
                }
            } else {
                node_coef<Real, UM>(ar, xo + e, c);
            }
            if (a.has_src) {
                const Real R = ((PRE ? rf[e] : (ar.rfield ? ar.rfield[xo + e] : a.R)) * a.src_mult) * su;
#pragma unroll
                for (int i = 0; i < Q; ++i) d[e][i] += R * Real(weight(i)) * (Real(1) + c.ex[i]);
            }
            NodeOut<Real> o;
            collide<Real, UM, false, sizeof(ST) == 4, sizeof(ST) != 2>(d[e], c, a.phi_ref * su, a.eps * su, a.tau2,
                                                                       a.root_rho, post[e], o);
            if (ar.lam_rec) {
                ar.lam_rec[xo + e] = o.lam;
                ar.br_rec[xo + e] = uint8_t(o.branch);
            }
            if (a.counters) {
                const unsigned slot = blockIdx.y + gridDim.y * blockIdx.z;
                if (o.branch != 255) atomicAdd(a.counters + cnt_index(0, slot), 1ull);
                if (!isfinite(o.dphi)) atomicAdd(a.counters + cnt_index(2, slot), 1ull);
                if (o.guard) atomicAdd(a.counters + cnt_index(3, slot), 1ull);
            }
            Real mass = o.dphi;
            if (ABB) {
                // a branch, not selects: only the first and the last wavefront of a row hold
                // a wall node
                const bool lo = lo_wall && e == 0, hi = hi_wall && e == V - 1;
                if (lo || hi)
                    reflect_at_walls(post[e], lo, hi, a.phi_lo * su, a.phi_hi * su, a.phi_ref * su, mass);
            }
            if constexpr (RS) store_rounding<ST, SU>(post[e], a, uint32_t(kr + xo + e), mass);
            if (SU && rest32) post[e][0] *= a.scale;
        }
    }
    if constexpr (W > 1) {
        // the first and last lane of every wavefront publish the values leaving the wave
        if (active && (lane == 0 || lane == 63)) {
#pragma unroll
            for (int i = 1; i < Q; ++i)
                if (cx(i) > 0 && lane == 63) xfer[threadIdx.y][w][i] = post[V - 1][i];
                else if (cx(i) < 0 && lane == 0) xfer[threadIdx.y][w][i] = post[0][i];
        }
        __syncthreads();
        if (!active) return;
    }
    // RS: store_rounding leaves the 16-bit values in storage units, stored unscaled
    const Real st_inv = (RS || SU) ? Real(1) : a.inv_scale;
    // push streaming: rows y +- 1, z +- 1 (periodic); x shift by rotation within the row
    const int ym = (y == 0) ? ny - 1 : y - 1, yp = (y == ny - 1) ? 0 : y + 1;
    const int zm = (z == 0) ? nz - 1 : z - 1, zp = (z == nz - 1) ? 0 : z + 1;
    const int ry[3] = {ym, y, yp};
    const int rz[3] = {zm * ny, z * ny, zp * ny};
    const int wl = (w == 0) ? W - 1 : w - 1, wr = (w == W - 1) ? 0 : w + 1;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        Real out[V];
        if (cx(i) == 0) {
#pragma unroll
            for (int e = 0; e < V; ++e) out[e] = post[e][i];
        } else if (cx(i) > 0) {
            out[0] = wave_rotate<1>(post[V - 1][i]);
            if (W > 1 && lane == 0) out[0] = xfer[threadIdx.y][wl][i];
#pragma unroll
            for (int e = 1; e < V; ++e) out[e] = post[e - 1][i];
        } else {
#pragma unroll
            for (int e = 0; e < V - 1; ++e) out[e] = post[e + 1][i];
            out[V - 1] = wave_rotate<-1>(post[0][i]);
            if (W > 1 && lane == 63) out[V - 1] = xfer[threadIdx.y][wr][i];
        }
        ST* drow = dst + size_t(rz[cz(i) + 1] + ry[cy(i) + 1]) * re;
        if constexpr (sizeof(ST) == 2) {
            if (i == 0 && rest32) {
                VecIO<float, V>::store(reinterpret_cast<float*>(drow) + xo, out, 1.0f);
                continue;
            }
        }
        ST* p = drow + run_offset(i, nx, rest32) + xo;
        if (ABB && ((cx(i) > 0 && lo_wall) || (cx(i) < 0 && hi_wall))) {
            // the wrapped element belongs to the wall node of the destination row, which
            // writes it itself: store the other V - 1 elements one by one
            const int skip = cx(i) > 0 ? 0 : V - 1;
#pragma unroll
            for (int e = 0; e < V; ++e)
                if (e != skip) Store<ST>::put(p + e, out[e], st_inv);
        } else {
            IO::store(p, out, st_inv);
        }
    }
    if (ABB && (lo_wall || hi_wall)) {
        // populations reflected at a Dirichlet plane (already turned into their opposite
        // by reflect_at_walls) stay at the wall node
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            if (lo_wall && cx(i) == -1) pop_put<ST>(dst, opp(i), r, xo, nx, post[0][i], rest32, st_inv);
            if (hi_wall && cx(i) == 1) pop_put<ST>(dst, opp(i), r, xo + V - 1, nx, post[V - 1][i], rest32, st_inv);
        }
    }
}

// Whether the row-vector kernel takes the XCD slab order (xcd_block). Measured on MI355X
// with every form on the decay (256^3), porous (384^3) and field (512^3) workloads: handing
// each XCD one contiguous eighth of the grid pays once a plane of the lattice moves more
// than about 28 MiB per step (field workload 512^3: FP64 +3 %, FP32 +8 %, the 16-bit forms
// at 29-30 MiB per plane +1-3 %; porous 384^3 FP64 +6 %), and costs 1-4 % well below that
// (the 256^3 decay in FP32 and 16-bit forms, 5-10 MiB), where the natural order's working
// set already fits each XCD's caches.
static int xcd_remap_for(const elbm_lattice* h, unsigned gy, unsigned gz) {
    if (gy % 8 != 0 || gz % 8 != 0) return 0;
    const int rb = real_bytes(h->cfg.precision);
    double node = 2.0 * double(elbm_population_bytes(h)) / double(h->n);
    node += h->t_field_mode == 1 ? 6.0 * rb : (h->t_field_mode == 2 ? 1.0 : 0.0);
    node += h->u_mode == 2 ? 3.0 * rb : 0.0;
    node += h->r_mode == 2 ? 1.0 * rb : 0.0;
    const double plane = node * double(h->cfg.nx) * double(h->cfg.ny);
    return plane >= 28.0 * 1024 * 1024 ? 1 : 0;
}

template <class ST, int UM, int V, int W>
static void launch_vec(const elbm_lattice* h, const StepArgs<typename Store<ST>::Real>& a_in) {
    constexpr int ROWS = (W == 3 || W > 4) ? 1 : 4 / W;
    const dim3 block(64 * W, ROWS, 1);
    const dim3 grid(1, (h->cfg.ny + ROWS - 1) / ROWS, h->cfg.nz);
    StepArgs<typename Store<ST>::Real> a = a_in;
    a.xcd_remap = xcd_remap_for(h, grid.y, grid.z);
    const bool rs = sizeof(ST) == 2 && (a.rest32 || a.sround);
    if (rs) {
        if constexpr (sizeof(ST) == 2) {
            if (a.abb)
                hipLaunchKernelGGL((k_step_vec<ST, UM, V, W, true, true>), grid, block, 0, h->stream, a);
            else
                hipLaunchKernelGGL((k_step_vec<ST, UM, V, W, false, true>), grid, block, 0, h->stream, a);
        }
    } else if (a.abb) {
        hipLaunchKernelGGL((k_step_vec<ST, UM, V, W, true, false>), grid, block, 0, h->stream, a);
    } else {
        hipLaunchKernelGGL((k_step_vec<ST, UM, V, W, false, false>), grid, block, 0, h->stream, a);
    }
}

template <class ST, int UM, int V>
static void launch_vec_w(const elbm_lattice* h, const StepArgs<typename Store<ST>::Real>& a, int W) {
    switch (W) {
        case 1: launch_vec<ST, UM, V, 1>(h, a); break;
        case 2: launch_vec<ST, UM, V, 2>(h, a); break;
        case 3: launch_vec<ST, UM, V, 3>(h, a); break;
        case 4: launch_vec<ST, UM, V, 4>(h, a); break;
        case 5: launch_vec<ST, UM, V, 5>(h, a); break;
        case 6: launch_vec<ST, UM, V, 6>(h, a); break;
        case 7: launch_vec<ST, UM, V, 7>(h, a); break;
        default: launch_vec<ST, UM, V, 8>(h, a); break;
    }
}

// Nodes per lane chosen when the flags set no width (0: one-node-per-thread kernel), the
// fastest measured on MI355X (256^3 decay with uniform coefficients, 384^3 porous with a
// per-node tensor field or material table, 512^3 with per-node tensor, velocity and source
// fields; same-box sweeps):
//  - 16-bit forms: 4 nodes (8 bytes) per lane, 2 with a velocity field (4 nodes: 34 %
//    slower there, 1 node: 1-6 %); on 384-node rows this halves to 2;
//  - FP32: 1 node per lane (field workload: 4.16 vs 4.27 ms with 2), except on 384-node
//    rows, where 1 would make a block of 6 wavefronts: there 2 (3 wavefronts; porous 384^3
//    1.0 % faster with the material table, 1.5 % with the tensor field, same box);
//  - FP64: 1 node per lane with uniform coefficients, 2 with a per-node tensor or velocity
//    (porous: 3.02 vs 3.75 ms; field workload: 10.1 ms, against 12.1 ms with 1 and
//    11.0 ms for the one-node-per-thread kernel).
// A return of 0 would select the one-node-per-thread kernel.
template <class ST>
static int auto_vector_width(bool tfield, bool ufield, int nx) {
    if (sizeof(ST) == 2) return ufield ? 2 : 4;
    if (sizeof(ST) == 4) return nx == 6 * 64 ? 2 : 1;
    return (tfield || ufield) ? 2 : 1;
}

// Row-vector launch if the row shape allows it: nx = 64 V W with 1 <= W <= 8;
// (flags >> 4) & 0xF sets the width. Without an explicit width, auto_vector_width's choice,
// or the nearest width (smaller first) that fits the row.
template <class ST, int UM>
static bool try_launch_vec(const elbm_lattice* h, const StepArgs<typename Store<ST>::Real>& a) {
    const int nx = h->cfg.nx;
    int V = (h->cfg.flags >> ELBM_VECTOR_WIDTH_SHIFT) & 0xF;
    if (V == 0) {
        const int pref = auto_vector_width<ST>(a.tfield != nullptr, a.ufield != nullptr, nx);
        if (pref == 0) return false;
        const int vmax = sizeof(ST) == 8 ? 2 : 4;
        const int order[5] = {pref, pref / 2, pref / 4, pref * 2, pref * 4};
        for (int c : order) {
            if (c < 1 || c > vmax || nx % (64 * c) != 0 || nx / (64 * c) > 8) continue;
            V = c;
            break;
        }
        if (V == 0) return false;
    }
    if (sizeof(ST) == 8 && V > 2) return false;
    if (V != 1 && V != 2 && V != 4) return false;
    if (nx % (64 * V) != 0) return false;
    const int W = nx / (64 * V);
    if (W < 1 || W > 8) return false;
    if (V == 1) launch_vec_w<ST, UM, 1>(h, a, W);
    else if (V == 2) launch_vec_w<ST, UM, 2>(h, a, W);
    else if constexpr (sizeof(ST) != 8) launch_vec_w<ST, UM, 4>(h, a, W);
    return true;
}

template <class ST, int UM, bool ABB>
__global__ __launch_bounds__(256) void k_adjoint(const StepArgs<typename Store<ST>::Real> a) {
    using Real = typename Store<ST>::Real;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= a.nx || y >= a.ny) return;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int nxy = nx * ny;
    const int k = z * nxy + y * nx + x;
    const ST* state = static_cast<const ST*>(a.src);

    // gather dL/dpost from the destinations of the push (transpose of streaming)
    const int xm = (x == 0) ? nx - 1 : x - 1, xp = (x == nx - 1) ? 0 : x + 1;
    const int ym = (y == 0) ? ny - 1 : y - 1, yp = (y == ny - 1) ? 0 : y + 1;
    const int zm = (z == 0) ? nz - 1 : z - 1, zp = (z == nz - 1) ? 0 : z + 1;
    const int ox[3] = {xm, x, xp};
    const int oy[3] = {ym * nx, y * nx, yp * nx};
    const int oz[3] = {zm * nxy, z * nxy, zp * nxy};
    Real ph[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const bool wall = ABB && ((cx(i) == 1 && x == nx - 1) || (cx(i) == -1 && x == 0));
        if (wall) {
            ph[i] = -a.adj_in[(size_t)opp(i) * a.n + k];
        } else {
            const int dk = oz[cz(i) + 1] + oy[cy(i) + 1] + ox[cx(i) + 1];
            ph[i] = a.adj_in[(size_t)i * a.n + dk];
        }
    }

    // the saved state is read once per reverse step: nontemporal loads
    Real d[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const ST* p = state + pop_offset(i, z * ny + y, x, nx, 0);
        if constexpr (sizeof(ST) == 2) d[i] = Store<ST>::load(p, a.scale);
        else d[i] = __builtin_nontemporal_load(p);
    }
    NodeCoef<Real> c;
    node_coef<Real, UM>(a, k, c);
    if (a.has_src) {
        const Real R = (a.rfield ? a.rfield[k] : a.R) * a.src_mult;
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] += R * Real(weight(i)) * (Real(1) + c.ex[i]);
    }
    Real dd[Q], tg[6];
    collide_vjp<Real>(d, c, a.phi_ref, a.eps, a.tau2, a.lam_in[k], int(a.br_in[k]), ph, dd, tg);
    // dL/dg_t and dL/dT are written once per reverse step, whole lines: nontemporal
#pragma unroll
    for (int i = 0; i < Q; ++i) __builtin_nontemporal_store(dd[i], a.adj_out + (size_t)i * a.n + k);
    add_t6(a.t_grad, k, tg);
}

// ------------------------------------------------------------------------------------------
// Host side
// ------------------------------------------------------------------------------------------
template <class ST, int UM>
static hipError_t step_t(const elbm_lattice* h, const void* src, void* dst, double src_mult,
                         void* lam_rec, uint8_t* br_rec) {
    using Real = typename Store<ST>::Real;
    StepArgs<Real> a = make_args<Real>(h, src_mult);
    a.src = src;
    a.dst = dst;
    a.lam_rec = static_cast<Real*>(lam_rec);
    a.br_rec = br_rec;
    // row-vector kernel: rows of 64 V W nodes, closed-form amplitude
    if (h->cfg.root_rho < 0 && !(h->cfg.flags & ELBM_FLAG_SCALAR_KERNEL) &&
        try_launch_vec<ST, UM>(h, a))
        return hipGetLastError();
    dim3 grid, block;
    grid_for(h, &grid, &block);
    const bool root = h->cfg.root_rho >= 0, abb = a.abb != 0;
    const bool rs = sizeof(ST) == 2 && (a.rest32 || a.sround);
    if (rs) {
        if constexpr (sizeof(ST) == 2) {
            if (root && abb)
                hipLaunchKernelGGL((k_step<ST, UM, true, true, true>), grid, block, 0, h->stream, a);
            else if (root)
                hipLaunchKernelGGL((k_step<ST, UM, true, false, true>), grid, block, 0, h->stream, a);
            else if (abb)
                hipLaunchKernelGGL((k_step<ST, UM, false, true, true>), grid, block, 0, h->stream, a);
            else
                hipLaunchKernelGGL((k_step<ST, UM, false, false, true>), grid, block, 0, h->stream, a);
        }
    } else if (root && abb) {
        hipLaunchKernelGGL((k_step<ST, UM, true, true, false>), grid, block, 0, h->stream, a);
    } else if (root) {
        hipLaunchKernelGGL((k_step<ST, UM, true, false, false>), grid, block, 0, h->stream, a);
    } else if (abb) {
        hipLaunchKernelGGL((k_step<ST, UM, false, true, false>), grid, block, 0, h->stream, a);
    } else {
        hipLaunchKernelGGL((k_step<ST, UM, false, false, false>), grid, block, 0, h->stream, a);
    }
    return hipGetLastError();
}

template <class ST>
static hipError_t step_u(const elbm_lattice* h, const void* src, void* dst, double m, void* lr,
                         uint8_t* br) {
    switch (h->u_mode) {
        case 0: return step_t<ST, 0>(h, src, dst, m, lr, br);
        case 1: return step_t<ST, 1>(h, src, dst, m, lr, br);
        default: return step_t<ST, 2>(h, src, dst, m, lr, br);
    }
}

template <class ST, int UM>
static hipError_t adj_t(const elbm_lattice* h, const void* state, double src_mult, const void* lam,
                        const uint8_t* br, const void* adj_in, void* adj_out, void* t_grad) {
    using Real = typename Store<ST>::Real;
    StepArgs<Real> a = make_args<Real>(h, src_mult);
    a.src = state;
    a.counters = nullptr;
    a.lam_in = static_cast<const Real*>(lam);
    a.br_in = br;
    a.adj_in = static_cast<const Real*>(adj_in);
    a.adj_out = static_cast<Real*>(adj_out);
    a.t_grad = static_cast<Real*>(t_grad);
    dim3 grid, block;
    grid_for(h, &grid, &block, 256);  // gathers and local writes: rows may be split
    if (a.abb)
        hipLaunchKernelGGL((k_adjoint<ST, UM, true>), grid, block, 0, h->stream, a);
    else
        hipLaunchKernelGGL((k_adjoint<ST, UM, false>), grid, block, 0, h->stream, a);
    return hipGetLastError();
}

template <class ST>
static hipError_t adj_u(const elbm_lattice* h, const void* s, double m, const void* l,
                        const uint8_t* b, const void* ai, void* ao, void* tg) {
    switch (h->u_mode) {
        case 0: return adj_t<ST, 0>(h, s, m, l, b, ai, ao, tg);
        case 1: return adj_t<ST, 1>(h, s, m, l, b, ai, ao, tg);
        default: return adj_t<ST, 2>(h, s, m, l, b, ai, ao, tg);
    }
}

}  // namespace elbm
