// HIP kernels of the reactive two-lattice lattice-Boltzmann step for gfx950.
//
// One time step (Falcucci et al., Appendix "Numerical Method"), two launches:
//   k_front      the sputtering boundary condition: every catalytic node k
//                takes In(k) = sum_j f*_j(k - c_j) over its active links
//                (first line of the sputtering equations; the sweep that
//                produced those populations summed it), accumulates it and
//                stores the re-emission (1 - p_S^R) In(k) scale(k); in the same
//                launch, the fixed-order FP64 reductions of the two previous
//                steps;
//   k_sweep_c /  fused pull-streaming + BGK collision of both lattices,
//   k_sweep      Eq. LBE with the second-order equilibrium, Guo body force on
//                the carrier, halfway bounce-back at solid links, the reactive
//                pull at catalytic sources and the reservoir planes; one lane
//                per gas node (k_sweep_c) or per voxel of a 64-voxel chunk.
//
// Storage: populations of gas nodes only, in (z, y, x) order, one array per
// direction whose element n is the pair (carrier, reactant) of node n, each
// as the normalised deviation h_i = f_i / w_i - rho_ref (rho_ref = rho0 for
// the carrier, c_ref for the reactant).  A gas neighbour's storage index is
// its chunk base plus a popcount of the chunk's gas bits, so no per-node
// neighbour table is read, only the 32-byte chunk records of the nine source
// rows.  Memory traffic is therefore close to 2 x 38 populations per gas node.

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "fixed_point.h"
#include "lbm_internal.h"

namespace lbmk {
namespace {

// Storage order of the direction arrays inside a lattice: the rest
// population first, then each velocity next to its opposite (i, opp(i)), so a
// pull and its bounce-back alternative share one base.
__host__ __device__ constexpr int dslot(int i) { return i == 0 ? 0 : (i <= 9 ? 2 * i - 1 : 2 * (i - 9)); }
__host__ __device__ constexpr int pair_slot(int i) { return i == 0 ? 0 : 2 * (i <= 9 ? i : i - 9) - 1; }

// ------------------------------------------------------------ storage --
template <int ST>
struct Store;
template <>
struct Store<ST_F32> {
    using S = float;
    using P = float __attribute__((ext_vector_type(2)));  // carrier and reactant of one direction
    using T = float;
    __device__ static T cv(S v) { return v; }
    __device__ static S enc(T v) { return v; }
    __device__ static T ld(const S *p) { return *p; }
    __device__ static void st(S *p, T v) { *p = v; }
    static constexpr bool ROUNDS = false;
    __device__ static P enc2(T c, T r, uint32_t, uint32_t) { return P{c, r}; }
    __device__ static S enc1(T v, uint32_t) { return v; }
};
template <>
struct Store<ST_F16> {
    using S = _Float16;
    using P = _Float16 __attribute__((ext_vector_type(2)));
    using T = float;
    __device__ static T cv(S v) { return static_cast<float>(v); }
    __device__ static T ld(const S *p) { return static_cast<float>(*p); }
    __device__ static S enc(T v) { return static_cast<_Float16>(v); }  // round to nearest even
    __device__ static void st(S *p, T v) { *p = enc(v); }
    // rounded by the word w (see lbmfx::round_words): nearest or stochastic
    static constexpr bool ROUNDS = true;
    // each conversion writes one half of its operand and keeps the other:
    // starting from the bits of c (whose register is free after the call)
    // spares a register clear per pair, and both halves are overwritten
    __device__ static P enc2(T c, T r, uint32_t wc, uint32_t wr) {
        P v = __builtin_bit_cast(P, c);
        v = __builtin_amdgcn_cvt_sr_f16_f32(v, c, wc, false);
        v = __builtin_amdgcn_cvt_sr_f16_f32(v, r, wr, true);
        return v;
    }
    __device__ static S enc1(T x, uint32_t w) {
        P v = __builtin_bit_cast(P, x);
        v = __builtin_amdgcn_cvt_sr_f16_f32(v, x, w, false);
        return v.x;
    }
};
template <>
struct Store<ST_BF16> {
    using S = uint16_t;
    using P = uint16_t __attribute__((ext_vector_type(2)));
    using T = float;
    __device__ static T cv(S v) { return __uint_as_float(uint32_t(v) << 16); }
    __device__ static T ld(const S *p) { return __uint_as_float(uint32_t(*p) << 16); }
    __device__ static S enc(T v) {
        const uint32_t u = __float_as_uint(v);
        const uint32_t rounded = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;  // round to nearest even
        return (u & 0x7fffffffu) > 0x7f800000u ? uint16_t((u >> 16) | 0x40u) : uint16_t(rounded);  // NaN stays NaN
    }
    __device__ static void st(S *p, T v) { *p = enc(v); }
    static constexpr bool ROUNDS = true;
    using B2 = __bf16 __attribute__((ext_vector_type(2)));
    __device__ static P enc2(T c, T r, uint32_t wc, uint32_t wr) {
        B2 v = __builtin_bit_cast(B2, c);  // both halves overwritten (see Store<ST_F16>)
        v = __builtin_amdgcn_cvt_sr_bf16_f32(v, c, wc, false);
        v = __builtin_amdgcn_cvt_sr_bf16_f32(v, r, wr, true);
        return __builtin_bit_cast(P, v);
    }
    __device__ static S enc1(T x, uint32_t w) {
        B2 v = __builtin_bit_cast(B2, x);
        v = __builtin_amdgcn_cvt_sr_bf16_f32(v, x, w, false);
        return __builtin_bit_cast(P, v).x;
    }
};
template <>
struct Store<ST_F64> {
    using S = double;
    using P = double __attribute__((ext_vector_type(2)));
    using T = double;
    __device__ static T cv(S v) { return v; }
    __device__ static S enc(T v) { return v; }
    __device__ static T ld(const S *p) { return *p; }
    __device__ static void st(S *p, T v) { *p = v; }
    static constexpr bool ROUNDS = false;
    __device__ static P enc2(T c, T r, uint32_t, uint32_t) { return P{c, r}; }
    __device__ static S enc1(T v, uint32_t) { return v; }
};

// Physical parameters in the compute type.
template <typename T>
struct PhysK {
    T om_c, om_r;     // 1 / tau
    T guo;            // 1 - 1 / (2 tau_gas)
    T fx, fy, fz;     // body force
    T rref, cref;     // storage shifts
    T h_inlet;        // c_inlet - c_ref: normalised inlet ghost population
    T keep;           // 1 - p_stick
    T a_r, a_p;       // product re-emission: p p_S^R of the reactant, 1 - p_S^P of the product
    T sigma;          // diffuse fraction of the carrier's wall reflection
    T h0c, h0r;       // initial state, normalised: rho0 - rho_ref, c0 - c_ref
    T usx, us3;       // reference flow U of the carrier's shifted form (store_ux) and 3 U
    double c_in;      // reservoir concentration (influx tally)
    double in_scale, in_unscale;  // fixed-point scale of the In(k) sums and its inverse
    int32_t sputter, coupling, species_x;
    uint32_t seed_lo, seed_hi, step_ctr;  // STOCHASTIC draws
    // 16-bit stores: stochastic rounding on (sr), keys of this launch's
    // rounding words for the population stores and the emission stores
    uint32_t sr, sr_key, sr_key_e;
};

template <typename T>
PhysK<T> to_kernel(const Physics &p) {
    PhysK<T> k;
    k.om_c = T(1.0 / p.tau_gas);
    k.om_r = T(1.0 / p.tau_species);
    k.guo = T(1.0 - 0.5 / p.tau_gas);
    k.fx = T(p.force[0]);
    k.fy = T(p.force[1]);
    k.fz = T(p.force[2]);
    k.rref = T(p.rho_ref);
    k.cref = T(p.c_ref);
    k.h_inlet = T(p.c_inlet - p.c_ref);
    k.keep = T(1.0 - p.p_stick);
    k.a_r = T(p.p * p.p_stick);
    k.a_p = T(1.0 - p.p_stick_product);
    k.sigma = T(p.wall_diffuse);
    k.h0c = T(p.rho0 - p.rho_ref);
    k.h0r = T(p.c0 - p.c_ref);
    k.usx = T(p.store_ux);
    k.us3 = T(3.0 * p.store_ux);
    k.c_in = p.c_inlet;
    k.in_scale = p.in_scale;
    k.in_unscale = p.in_unscale;
    k.sputter = p.sputter;
    k.coupling = p.coupling;
    k.species_x = p.species_x;
    k.seed_lo = uint32_t(p.seed);
    k.seed_hi = uint32_t(p.seed >> 32);
    k.step_ctr = p.step_ctr;
    k.sr = p.rounding == ROUND_STOCHASTIC && storage_bytes(p.storage) == 2;
    k.sr_key = lbmfx::round_key(p.step_ctr, p.seed, 0u);
    k.sr_key_e = lbmfx::round_key(p.step_ctr, p.seed, 1u);
    return k;
}

// ------------------------------------------------- random sputtering --
// STOCHASTIC: each arrival at interface node k along active link j leaves
// whole along one of the b(k) exit directions {opp(j')}, picked with
// probability 1/b by Philox4x32-10 (Salmon et al., SC 2011): key (seed low,
// seed high), counter (step, voxel index of k, code(j), 0), first output word
// r, exit number floor(r b / 2^32) in ascending code order, where code(c) =
// 9 (c_x + 1) + 3 (c_y + 1) + (c_z + 1) labels a velocity independently of
// the direction numbering.
__host__ __device__ constexpr int vcode(int i) { return 9 * (CX[i] + 1) + 3 * (CY[i] + 1) + (CZ[i] + 1); }

// Directions 1..18 in ascending velocity code.
struct CodeOrder {
    int d[18];
};
__host__ __device__ constexpr CodeOrder code_order() {
    CodeOrder o{};
    int n = 0;
    for (int code = 0; code < 27; ++code)
        for (int i = 1; i < 19; ++i)
            if (vcode(i) == code) o.d[n++] = i;
    return o;
}
constexpr CodeOrder CODE_ORDER = code_order();

__device__ __forceinline__ uint32_t philox_first(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                 uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return c0;
}

// The exit direction (library numbering) of an arrival along the link with
// velocity code `code` at the interface node with voxel index vox and
// active-link mask `mask`.
__device__ __forceinline__ int random_exit(uint32_t step, uint32_t seed_lo, uint32_t seed_hi, uint32_t vox,
                                           uint32_t mask, uint32_t code) {
    const uint32_t b = uint32_t(__popc(mask));
    const uint32_t r = philox_first(step, vox, code, 0u, seed_lo, seed_hi);
    const uint32_t pick = uint32_t((uint64_t(r) * b) >> 32);
    int e = 0;
    uint32_t n = 0;
#pragma unroll
    for (int t = 0; t < 18; ++t) {
        const int d = CODE_ORDER.d[t];
        const bool exit = (mask >> opp(d)) & 1u;
        e = (exit && n == pick) ? d : e;
        n += exit ? 1u : 0u;
    }
    return e;
}

// One term of an In(k) sum, f*_j = w_j (h_j + c_ref) of the stored value, in
// fixed point (lbmfx::term: MAGIC_BITS + round(term * 2^S), or a poison
// pattern the reader reports as non-finite).  The sums add bit patterns; the
// reader subtracts b(k) * MAGIC_BITS.
constexpr unsigned long long MAGIC_BITS = lbmfx::MAGIC_BITS;
template <typename T>
__device__ __forceinline__ unsigned long long in_term(T w, T h_stored, T cref, double scale) {
    return lbmfx::term(double(w * (h_stored + cref)), scale);
}

// ------------------------------------------------------------ helpers --
// Every buffer lives in device global memory; saying so lets the compiler use
// global (not flat) instructions also for pointers read from a batch record.
#define LBM_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ LBM_GLOBAL T *glb(T *p) {
    return (LBM_GLOBAL T *)(p);
}
// Element index of node n inside one slot of a population array (see
// Geometry::lay_ss / lay_bs); the slot adds s lay_ss elements.  n < 2^30, so
// n >> 6 and lay_bs fit the 24-bit multiplier.
__device__ __forceinline__ uint32_t node_elem(const Geometry &g, uint32_t n) {
    return __umul24(n >> 6, g.lay_bs) + (n & 63u);
}
__device__ __forceinline__ uint64_t slot_elem(const Geometry &g, int slot) { return uint64_t(uint32_t(slot)) * g.lay_ss; }

// Keep a selected value opaque to the optimizer (no instruction is emitted):
// stops it from folding a select into the address arithmetic and turning the
// select back into divergent branches.
__device__ __forceinline__ void opaque(uint32_t &v) { asm("" : "+v"(v)); }
// Same for a wave-uniform 64-bit value kept in a scalar register pair.
__device__ __forceinline__ uint64_t opaque_s(uint64_t v) {
    asm("" : "+s"(v));
    return v;
}

__device__ __forceinline__ uint32_t bits_below_lane(uint64_t m) {
    // number of set bits of m below this lane (lane = position within the chunk)
    return __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic block sum of NV values (256 threads = 4 waves), written by
// thread 0 to out[0..NV).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *out) {
    __shared__ double sh[4][NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[wave][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) glb(out)[k] = ((sh[0][k] + sh[1][k]) + sh[2][k]) + sh[3][k];
}

// The same for a block of one wavefront: lane 0 writes the wavefront's sums.
template <int NV>
__device__ __forceinline__ void wave_partials(double (&v)[NV], double *out) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if ((threadIdx.x & 63u) == 0u)
#pragma unroll
        for (int k = 0; k < NV; ++k) glb(out)[k] = v[k];
}

// Where a wavefront sits: which row and chunk, and this lane's node.
struct WaveUnit {
    int row, chunk, lane, x, y, z;
    bool valid;      // the unit exists
    bool active;     // this lane is a gas node
    uint32_t idx;    // storage index of this lane's node
};

__device__ __forceinline__ int xcd_block(int b, int nb) {
    // Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous range of rows so neighbouring rows share its L2.  The sweep
    // grids are padded to a multiple of 8 blocks; other grids keep their order.
    const int per = nb >> 3;
    if ((nb & 7) != 0 || per == 0) return b;
    return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ WaveUnit locate(const Geometry &g, uint32_t block) {
    // The traversal order (which x-row chunk each wave takes) is a host-built
    // table of codes y | z << 12 | chunk << 24, one per wave, read with one
    // scalar load.  `block` is the logical block (after the XCD remap).
    WaveUnit u;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const uint32_t unit = block * 4u + uint32_t(wave);
    u.valid = unit < g.units;
    const uint32_t code = glb(g.order)[u.valid ? unit : 0u];
    u.y = int(code & 0xfffu);
    u.z = int((code >> 12) & 0xfffu);
    u.chunk = int(code >> 24);
    u.row = u.z * g.ny + u.y;
    u.lane = int(threadIdx.x & 63);
    u.x = u.chunk * 64 + u.lane;
    const LBM_GLOBAL ChunkInfo &I = glb(g.chunks)[uint32_t(u.row) * uint32_t(g.W) + uint32_t(u.chunk)];
    const uint64_t fl = I.fluid;
    u.active = u.valid && u.x < g.nx && ((fl >> u.lane) & 1u);
    u.idx = I.base + bits_below_lane(fl);
    return u;
}

// Loads and stores at a wave-uniform base plus a 32-bit per-lane byte
// offset: the global memory instructions take the base in scalar registers,
// so no per-lane 64-bit address arithmetic is needed.
template <typename S>
__device__ __forceinline__ S ld_at(const S *base, uint32_t byte_off) {
    return *(const LBM_GLOBAL S *)((const LBM_GLOBAL char *)(base) + byte_off);
}
// One element of a direction array (carrier and reactant population) in a
// single load.  With 16-bit storage the loads bypass the cache allocation:
// every element is read once per sweep.  (Measured: the streaming form slows
// the FP32 sweep, whose row-edge lines are shared by two readers.)
template <int ST>
__device__ __forceinline__ typename Store<ST>::P ld_pop(const void *base, uint32_t byte_off) {
    using P = typename Store<ST>::P;
    const LBM_GLOBAL P *a = (const LBM_GLOBAL P *)((const LBM_GLOBAL char *)(base) + byte_off);
    if constexpr (sizeof(typename Store<ST>::S) == 2)
        return __builtin_nontemporal_load(a);
    else
        return *a;
}
template <int ST>
__device__ __forceinline__ typename Store<ST>::P pop_pair(typename Store<ST>::T c, typename Store<ST>::T r) {
    typename Store<ST>::P v;
    v.x = Store<ST>::enc(c);
    v.y = Store<ST>::enc(r);
    return v;
}
template <typename S>
__device__ __forceinline__ void st_at(S *base, uint32_t byte_off, S v) {
    *(LBM_GLOBAL S *)((LBM_GLOBAL char *)(base) + byte_off) = v;
}
// Streaming store: the populations written by a sweep are not read again
// before the next sweep, so they need not stay in the caches.  Used where
// every store of a wavefront covers whole lines (the node-compact sweep);
// the chunk sweep's partial-line stores lose write combining with it.
template <typename S>
__device__ __forceinline__ void st_stream(S *base, uint32_t byte_off, S v) {
    __builtin_nontemporal_store(v, (LBM_GLOBAL S *)((LBM_GLOBAL char *)(base) + byte_off));
}

// A population buffer: 19 slots (dslot(i)) of `stride` bytes each from
// `base` (stride = lay_ss elements); node n of a slot is element
// node_elem(n).  An element is the pair (carrier, reactant) of a gas node, so
// the common pull, where both lattices take the same source, is one load and
// the store of a direction one store.
// A direction's base address is formed in scalar registers where it is used
// (one 64-bit multiply-add), so the kernels do not hold 38 pointers in scalar
// registers.  (The create path guarantees that two direction arrays span
// less than 4 GiB, so the stride fits in 32 bits.)
struct Slots {
    const char *base;
    uint32_t stride, pad;
    __device__ __forceinline__ const void *p(int slot) const { return base + uint64_t(uint32_t(slot)) * stride; }
};
struct OutSlots {
    char *base;
    uint32_t stride, pad;
    __device__ __forceinline__ void *p(int slot) const { return base + uint64_t(uint32_t(slot)) * stride; }
};

// Template code of a sweep: the sputter mode, plus this flag for INFLOW, so
// the kernels of the other boundaries carry none of its code, and this one
// for the product lattice (node-compact sweep only).
constexpr int SP_INFLOW_FLAG = 4;
constexpr int SP_PRODUCT_FLAG = 8;
// and this one for a diffuse carrier wall (single-context sweeps only)
constexpr int SP_DIFFUSE_FLAG = 16;

// Diffuse carrier wall (Maxwell accommodation; lattice Boltzmann form of
// Ansumali and Karlin, Phys. Rev. E 66, 026311 (2002)): the populations a gas
// node pulls from solid sources (its own reversed populations, h = f/w -
// rho_ref) keep 1 - sigma of themselves and take sigma of the mass the node
// sent into the wall, spread as w_i: h_i += sigma (sum_s w_s h_s / sum_s w_s -
// h_i) over the solid-source directions s.
template <typename T>
__device__ __forceinline__ void diffuse_wall(T sigma, uint32_t solid_bits, T (&hC)[19]) {
    T m = 0, w = 0;
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        const bool s = (solid_bits >> i) & 1u;
        m += s ? wgt<T>(i) * hC[i] : T(0);
        w += s ? wgt<T>(i) : T(0);
    }
    const T mh = w > T(0) ? m / w : T(0);
#pragma unroll
    for (int i = 1; i < 19; ++i)
        if ((solid_bits >> i) & 1u) hC[i] = hC[i] + sigma * (mh - hC[i]);
}

// Reference flow of the carrier (lbm_bc.store_ux = U): the carrier is stored
// and relaxed in the shifted form h'_i = h_i - 3 c_ix U, its deviation less
// the part of the equilibrium linear in a reference x-velocity.  In a flow
// near U these values are small, so their rounding (storage and arithmetic)
// is too.  The form is exact algebra: sum_i w_i h'_i = sum_i w_i h_i and
// sum_i w_i c_ix h'_i = sum_i w_i c_ix h_i - U (moments add U back), and
// the equilibrium takes the same shift (collide).  Uniform branches: nothing
// runs when U is 0.  FP32 storage takes no reference flow (the host keeps U
// at 0 there), so its pulls carry none of this code.
//
// After a pull, direction i holds population i of a gas source (already in
// the shifted form of direction i) or, where the source is solid, the node's
// own opp(i), shifted as opp(i): c_ix us3 too high for direction i.  These
// steps take the bounced values down in two halves, so that between them
// they are true deviations (the diffuse wall mixes them there).
template <typename T>
__device__ __forceinline__ void bounced_half_shift(const PhysK<T> &ph, uint32_t solid_bits, T (&hC)[19]) {
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        if (CX[i] == 0) continue;
        if ((solid_bits >> i) & 1u) hC[i] -= T(CX[i]) * ph.us3;
    }
}
// true deviations -> shifted form (initial state)
template <typename T>
__device__ __forceinline__ void carrier_shift(const PhysK<T> &ph, T (&hC)[19]) {
    if (ph.us3 != T(0)) {
#pragma unroll
        for (int i = 1; i < 19; ++i)
            if (CX[i] != 0) hC[i] -= T(CX[i]) * ph.us3;
    }
}
// shifted form -> true deviations (population readback)
template <typename T>
__device__ __forceinline__ void carrier_unshift(const PhysK<T> &ph, T (&hC)[19]) {
    if (ph.us3 != T(0)) {
#pragma unroll
        for (int i = 1; i < 19; ++i)
            if (CX[i] != 0) hC[i] += T(CX[i]) * ph.us3;
    }
}

// The product lattice as the sweep sees it: P population buffers (one
// population per element, same slot order as the pair buffers), E_P(k),
// In_P(k) and the sweep's three P partials per block.
template <int ST>
struct ProdK {
    Slots in;
    OutSlots out;
    const typename Store<ST>::S *emit;
    unsigned long long *inacc;
    double *part;
};

// INFLOW species x-boundary: the inlet ghost populations pulled by a node at
// x = 0 (directions with c_x = +1) are the equilibrium of c_in moving with the
// carrier velocity of that node, u = (j_C + F/2) / rho_C from the carrier
// populations it has just pulled.
template <typename T>
__device__ __forceinline__ void weighted_moments(const T (&h)[19], T &d, T &jx, T &jy, T &jz);
template <typename T>
__device__ __forceinline__ void inflow_ghost(const PhysK<T> &ph, const T (&hC)[19], T (&hR)[19]) {
    T d, jx, jy, jz;
    weighted_moments(hC, d, jx, jy, jz);
    const T inv = T(1) / (ph.rref + d);
    // the carrier is in its shifted form (reference flow usx)
    const T ux = (jx + ph.usx + T(0.5) * ph.fx) * inv, uy = (jy + T(0.5) * ph.fy) * inv, uz = (jz + T(0.5) * ph.fz) * inv;
    const T uu = ux * ux + uy * uy + uz * uz;
    const T cin = T(ph.c_in);
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        if (CX[i] != 1) continue;
        const T cu = ux + T(CY[i]) * uy + T(CZ[i]) * uz;
        hR[i] = cin * (T(1) + T(3) * cu + T(4.5) * cu * cu - T(1.5) * uu) - ph.cref;
    }
}

// Directions grouped by source row (cy, cz), so each row's chunk record is
// needed for one stretch of the pull only.
constexpr int ORDER[18] = {1, 10, 2, 4, 14, 11, 13, 5, 3, 6, 16, 12, 15, 7, 8, 9, 17, 18};

// Per-lane predicates of one pull direction, held as 64-bit lane masks
// (bit L = lane L of the wave) so that they are formed once per wave on the
// scalar unit and feed the vector selects directly.
__device__ __forceinline__ bool lane_in(uint64_t mask) { return __builtin_amdgcn_inverse_ballot_w64(mask); }

__device__ __forceinline__ uint32_t rank_of_mask(uint64_t m, uint32_t add) {
    // add + number of set bits of m below this lane
    return __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), add));
}

// Pull both lattices into registers: hC[i], hR[i] are the normalised
// populations of this node after streaming (the pre-collision state).
// kidx (LDS, may be null): receives, per direction i and lane, the
// interface index of the lane's source x - c_i (meaningful where it is an
// interface node), for the sweep's In(k) accumulation.
template <int ST, int SP>
__device__ __forceinline__ void pull(const Geometry &g, const PhysK<typename Store<ST>::T> &ph, const Slots &in,
                                     const typename Store<ST>::S *__restrict__ emit, const WaveUnit &u,
                                     typename Store<ST>::T (&hC)[19], typename Store<ST>::T (&hR)[19],
                                     uint32_t &cat_out, uint32_t *kidx = nullptr) {
    using T = typename Store<ST>::T;
    using S = typename Store<ST>::S;
    using P = typename Store<ST>::P;
    constexpr uint32_t SB = sizeof(S), PB = 2 * SB;
    const uint32_t nfp_b = in.stride;   // one slot, in bytes
    const bool reservoir = ph.species_x != XB_PERIODIC;  // inlet and outlet ghost planes
    // SP: the sputter mode (bits 0-1) and the INFLOW flag, fixed at compile
    // time for the sweeps, or -1 to read both from ph
    const int sputter = SP >= 0 ? (SP & 3) : ph.sputter;
    const bool inflow = SP >= 0 ? (SP & SP_INFLOW_FLAG) != 0 : ph.species_x == XB_INFLOW;
    const bool bounce = sputter == SP_BOUNCEBACK, uniform = sputter == SP_UNIFORM;
    const bool stoch = sputter == SP_STOCHASTIC;  // per-exit emission slots (already divided by w_i)
    const bool diffuse = SP >= 0 ? (SP & SP_DIFFUSE_FLAG) != 0 : ph.sigma != T(0);
    uint32_t solid_bits = 0;  // directions whose source is solid (the carrier reflects there)
    auto base = [&](int slot) { return in.p(slot); };
    const uint32_t own_b = node_elem(g, u.idx) * PB;
    // wave-uniform shape of the chunk
    const int nvalid = min(64, g.nx - 64 * u.chunk);
    const int last_lane = nvalid - 1;
    const bool first_chunk = u.chunk == 0, last_chunk = u.chunk == g.W - 1;
    const uint64_t lane0 = 1ull, lane_last = 1ull << last_lane;

    // Phase 1: every address, then every load (up to 42 in flight per lane).
    P pc[19];
    S re[19], ro[19];
    uint32_t cat_bits = 0;
    pc[0] = ld_pop<ST>(base(dslot(0)), own_b);
    // the nine source rows (wave-uniform): chunk record and first voxel
    const LBM_GLOBAL ChunkInfo *recs[9];
#pragma unroll
    for (int cy = -1; cy <= 1; ++cy) {
        int ys = u.y - cy;
        ys = ys < 0 ? ys + g.ny : (ys >= g.ny ? ys - g.ny : ys);
#pragma unroll
        for (int cz = -1; cz <= 1; ++cz) {
            int zs = u.z - cz;
            zs = zs < 0 ? zs + g.nz : (zs >= g.nz ? zs - g.nz : zs);
            const uint32_t r = uint32_t(__builtin_amdgcn_readfirstlane(zs * g.ny + ys));
            recs[(cy + 1) * 3 + cz + 1] = glb(g.chunks) + (r * uint32_t(g.W) + uint32_t(u.chunk));
        }
    }
#pragma unroll
    for (int k = 0; k < 18; ++k) {
        const int i = ORDER[k];
        const int cx = CX[i];
        // source row of this direction and its chunk record
        const LBM_GLOBAL ChunkInfo &I = *recs[(CY[i] + 1) * 3 + CZ[i] + 1];
        // F / C: the source x - cx of each lane is gas / catalytic; rank: its
        // storage index when gas.
        // irank: the source's interface index when it is an interface node
        uint64_t F, C;
        uint32_t rank, irank;
        if (cx == 0) {
            F = I.fluid;
            C = I.cat;
            rank = rank_of_mask(I.fluid, I.base);
            irank = rank_of_mask(I.cat, I.ibase);
        } else if (cx == 1) {  // source x - 1; lane 0 takes the left neighbour of the chunk
            const uint32_t pv = I.prev;
            const uint32_t pf = pv >> 31, pc = (pv >> 30) & 1u;
            F = (I.fluid << 1) | pf;
            C = (I.cat << 1) | pc;
            rank = rank_of_mask(F, I.base - pf);
            irank = rank_of_mask(C, I.ibase - pc);
            if (first_chunk) {  // periodic wrap to x = nx - 1
                rank = lane_in(lane0) ? (pv & NB_IDX) : rank;
                irank = lane_in(lane0) ? (pv & NB_IDX) : irank;
            }
        } else {  // source x + 1; the last valid lane takes the right neighbour
            const uint32_t nv = I.next;
            F = (I.fluid >> 1) | (uint64_t(nv >> 31) << last_lane);
            C = (I.cat >> 1) | (uint64_t((nv >> 30) & 1u) << last_lane);
            rank = rank_of_mask(I.fluid >> 1, I.base + uint32_t(I.fluid & 1u));
            irank = rank_of_mask(I.cat >> 1, I.ibase + uint32_t(I.cat & 1u));
            if (last_chunk) {  // periodic wrap to x = 0
                rank = lane_in(lane_last) ? (nv & NB_IDX) : rank;
                irank = lane_in(lane_last) ? (nv & NB_IDX) : irank;
            }
        }
        // Direction i and opp(i) are adjacent arrays: one base, and the pull
        // or the bounce-back is an offset of 0 or nfp elements plus a node.
        const uint32_t half = dslot(i) < dslot(opp(i)) ? 0u : nfp_b;  // i's array inside the pair
        const uint32_t bb_b = own_b + (nfp_b - half);                   // own opp(i) entry
        const uint32_t pull_b = node_elem(g, rank) * PB + half;
        // both lattices from the gas source, or both bounced back
        pc[i] = ld_pop<ST>(base(pair_slot(i)), lane_in(F) ? pull_b : bb_b);
        solid_bits |= lane_in(F) ? 0u : (1u << i);
        // Reactant exceptions: the reservoir planes and catalytic sources.
        const uint64_t inlet = (reservoir && cx == 1 && first_chunk) ? lane0 : 0ull;
        const uint64_t outlet = (reservoir && cx == -1 && last_chunk) ? lane_last : 0ull;
        const uint64_t CAT = ~F & C & ~inlet & ~outlet;
        const uint64_t EMIT = bounce ? 0ull : CAT;
        // the outlet lane copies plane nx - 1 of the source row (bounce-back
        // where that voxel is solid)
        ro[i] = S(0);
        if (outlet)
            ro[i] = ld_at(static_cast<const S *>(base(pair_slot(i))),
                          (lane_in(outlet & I.fluid) ? node_elem(g, rank_of_mask(I.fluid, I.base)) * PB + half : bb_b) +
                              SB);
        // emission of a catalytic source, by interface index (element 0 when not used)
        re[i] = ld_at(emit, lane_in(EMIT) ? (stoch ? uint32_t(i - 1) * g.niface + irank : irank) * SB : 0u);
        if (kidx) kidx[(i - 1) * 256 + threadIdx.x] = irank;
        cat_bits |= lane_in(CAT) ? (1u << i) : 0u;
    }
    __builtin_amdgcn_sched_barrier(0);
    // Phase 2: decode and apply the reservoir and sputtering rules.  The inlet
    // lane takes the reservoir population w_i c_in (as stored).
    const T h_in = Store<ST>::cv(Store<ST>::enc(ph.h_inlet));
    hC[0] = Store<ST>::cv(pc[0].x);
    hR[0] = Store<ST>::cv(pc[0].y);
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        hC[i] = Store<ST>::cv(pc[i].x);
        T v = Store<ST>::cv(pc[i].y);
        if (CX[i] == 1 && reservoir && first_chunk) v = lane_in(lane0) ? h_in : v;
        if (CX[i] == -1 && reservoir && last_chunk) v = lane_in(lane_last) ? Store<ST>::cv(ro[i]) : v;
        const T e = Store<ST>::cv(re[i]);
        const T v_cat = bounce ? ph.keep * (v + ph.cref) - ph.cref : (uniform ? e * inv_wgt<T>(i) : e) - ph.cref;
        hR[i] = ((cat_bits >> i) & 1u) ? v_cat : v;
    }
    // the reference flow (none with FP32 storage, whose sweep is register bound)
    const bool shifted = ST != ST_F32 && ph.us3 != T(0);
    if constexpr (ST != ST_F32)
        if (shifted) bounced_half_shift(ph, solid_bits, hC);
    if (diffuse && solid_bits != 0u) diffuse_wall(ph.sigma, solid_bits, hC);
    if constexpr (ST != ST_F32)
        if (shifted) bounced_half_shift(ph, solid_bits, hC);
    if (inflow && first_chunk && lane_in(lane0)) inflow_ghost(ph, hC, hR);
    cat_out = cat_bits;
}

// The 64 consecutive gas nodes of a compact wavefront lie in a few
// consecutive (row, chunk) units of the lattice (at 256^3, porosity 0.61: at
// most 3 for 93 % of the wavefronts, at most 4 for 99.7 %), and
// the nine source-row records a lane needs are those of its unit shifted by
// the nine (c_y, c_z) classes.  When the wavefront spans at most WREC_UNITS
// units (host table g.wunits: first unit u0 and count nu), its lanes load all
// 9 x nu records once (one record per lane) and store each in the wavefront's
// LDS slice in a form that leaves each lane little work of its own (XRec
// below).  The records of the wavefront's own units (class 0) also give each
// lane its coordinates: lane `rank` lies in the last unit whose first gas
// node is at or before it, at the (rank - base)-th gas bit of that unit, so
// no per-node coordinate is read.  Called by every lane of a valid wavefront;
// returns false, with nothing loaded, when the wavefront spans more units.
// The node-compact sweep runs one wavefront per block: its lanes share no
// LDS or barrier with other wavefronts, so a wavefront that finishes early
// frees its slot without waiting for its neighbours.
// WREC_UNITS = 4 keeps the LDS of a block (records and kidx) within 1/24 of
// a CU's, so six wavefronts per SIMD fit.
constexpr uint32_t CTHREADS = 64;
constexpr uint32_t WREC_UNITS = 4;
// (c_y + 1) and (c_z + 1) of the nine classes, two bits each, class order as CYS / CZS
constexpr uint32_t CLS_CY1 = (1u << 0) | (2u << 2) | (0u << 4) | (1u << 6) | (1u << 8) | (2u << 10) | (2u << 12) |
                             (0u << 14) | (0u << 16);
constexpr uint32_t CLS_CZ1 = (1u << 0) | (1u << 2) | (1u << 4) | (2u << 6) | (0u << 8) | (2u << 10) | (0u << 12) |
                             (0u << 14) | (2u << 16);

// Bit index of the k-th (from 0) set bit of m (k < popcount(m)).
__device__ __forceinline__ uint32_t kth_set_bit(uint64_t m, uint32_t k) {
    uint32_t v = uint32_t(m), pos = 0u;
    uint32_t c = uint32_t(__popc(v));
    if (k >= c) {
        k -= c;
        v = uint32_t(m >> 32);
        pos = 32u;
    }
#pragma unroll
    for (uint32_t w = 16u; w >= 1u; w >>= 1) {
        c = uint32_t(__popc(v & ((1u << w) - 1u)));
        const bool up = k >= c;
        k -= up ? c : 0u;
        v = up ? v >> w : v;
        pos += up ? w : 0u;
    }
    return pos;
}

// One source-row record as the lanes read it.  E is the 66-bit window string
// of a chunk: E[0] the voxel left of the chunk (periodic), E[1 + b] voxel b
// of the chunk, and E[p] with p = min(64, nx - 64 chunk) + 1 the voxel right
// of its last voxel (periodic), held in three words; the gas (f) and
// interface (c) strings are kept apart.  A lane at chunk offset xl finds
// its three bits (x - 1, x, x + 1) at E[xl .. xl + 2], one funnel shift of
// words xl / 32 and xl / 32 + 1.  q[k] = base - E[0] + (set bits of E below
// bit 32 k), so the rank of x (the storage index of x if gas, of the next
// gas voxel otherwise) is q[k] + (set bits of word k below bit (xl + 1) %
// 32), k = (xl + 1) / 32: storage indices (and interface indices) run in (z,
// y, x) order, so within a row the gas neighbours of x are rank - 1 and rank
// + 1.  Only the periodic wrap of x needs the stored neighbours: pv (x = 0:
// the index of voxel nx - 1) and nv (x = nx - 1: the index of voxel 0).
// Words interleave as (E_f[k], q_f[k]) pairs so that both reads of a lane
// come as two-word LDS reads from one address.
struct XRec {
    uint32_t f[6];  // E_f[0], q_f[0], E_f[1], q_f[1], E_f[2], q_f[2]
    uint32_t c[6];  // the same for the interface string
    uint32_t pv, nv;  // storage / interface index of the periodic neighbours (NB_IDX bits)
};

struct WaveRecords {
    XRec rec[WREC_UNITS * 9];  // unit-major: rec[j * 9 + cls]
    uint64_t ufm[WREC_UNITS];  // gas mask of the wavefront's own unit j (class 0)
    uint32_t ubase[WREC_UNITS];
    uint32_t upos[WREC_UNITS];  // x of the unit's first voxel | y << 12 | z << 22
};

// trunc((n + 1/2) * inv): n / d for n < 2^26, d <= 2^12, inv = 1 / d in FP64
__device__ __forceinline__ uint32_t div_recip(uint32_t n, double inv) {
    return uint32_t(__builtin_fma(double(n), inv, 0.5 * inv));
}

// E string words and rank offsets of one mask (see XRec).
__device__ __forceinline__ void window_words(uint64_t m, uint32_t left, uint32_t right, uint32_t p, uint32_t base,
                                             uint32_t (&w)[6]) {
    uint64_t lo = (m << 1) | uint64_t(left);
    uint32_t hi = uint32_t(m >> 63);
    lo |= p < 64u ? uint64_t(right) << p : 0u;
    hi |= p >= 64u ? right << (p - 64u) : 0u;
    w[0] = uint32_t(lo);
    w[2] = uint32_t(lo >> 32);
    w[4] = hi;
    w[1] = base - left;
    w[3] = w[1] + uint32_t(__popc(w[0]));
    w[5] = w[3] + uint32_t(__popc(w[2]));
}

__device__ __forceinline__ bool wave_records(const Geometry &g, uint32_t w, uint32_t rank, bool active,
                                             WaveRecords &wr, uint32_t &wunit, uint32_t &pos) {
    const uint32_t wu = glb(g.wunits)[w];
    const uint32_t u0 = wu & ((1u << 26) - 1u), nu = wu >> 26;
    if (nu > WREC_UNITS) return false;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t ny = uint32_t(g.ny), nz = uint32_t(g.nz);
    if (lane < 9u * nu) {
        const uint32_t j = lane / 9u, cls = lane - 9u * j;
        const uint32_t u = u0 + j;
        const uint32_t row = div_recip(u, g.inv_W), chunk = u - row * uint32_t(g.W);
        const uint32_t zr = div_recip(row, g.inv_ny), yr = row - zr * ny;
        // source row of the class: (y - c_y, z - c_z), periodic
        const uint32_t cy1 = (CLS_CY1 >> (2u * cls)) & 3u, cz1 = (CLS_CZ1 >> (2u * cls)) & 3u;
        uint32_t ys = yr + ny + 1u - cy1, zs = zr + nz + 1u - cz1;
        ys = ys >= ny ? ys - ny : ys;
        ys = ys >= ny ? ys - ny : ys;
        zs = zs >= nz ? zs - nz : zs;
        zs = zs >= nz ? zs - nz : zs;
        const LBM_GLOBAL ChunkInfo &src = glb(g.chunks)[(zs * ny + ys) * uint32_t(g.W) + chunk];
        const uint64_t fm = src.fluid, cm = src.cat;
        const uint32_t pv = src.prev, nv = src.next, base = src.base;
        const uint32_t p = min(64u, uint32_t(g.nx) - 64u * chunk) + 1u;
        XRec &dst = wr.rec[lane];
        uint32_t wf[6], wc[6];
        window_words(fm, pv >> 31, nv >> 31, p, base, wf);
        window_words(cm, (pv >> 30) & 1u, (nv >> 30) & 1u, p, src.ibase, wc);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            dst.f[k] = wf[k];
            dst.c[k] = wc[k];
        }
        dst.pv = pv & NB_IDX;
        dst.nv = nv & NB_IDX;
        if (cls == 0u) {
            wr.ufm[j] = fm;
            wr.ubase[j] = base;
            wr.upos[j] = (chunk << 6) | (yr << 12) | (zr << 22);
        }
    }
    // the wavefront's LDS writes before its reads
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    uint32_t jj = 0u, kb = 0u;
    uint64_t fm = 0u;
#pragma unroll
    for (uint32_t j = 0; j < WREC_UNITS; ++j) {
        if (j < nu) {
            const uint64_t f = wr.ufm[j];
            const uint32_t b = wr.ubase[j];
            const bool here = f != 0u && b <= rank;
            jj = here ? j : jj;
            kb = here ? b : kb;
            fm = here ? f : fm;
        }
    }
    wunit = jj;
    pos = active ? wr.upos[jj] + kth_set_bit(fm, rank - kb) : 0u;
    return true;
}

// What a lane takes from one source row: its three gas and interface bits
// (x - 1, x, x + 1 in bits 0-2) and the ranks of x in the row's storage and
// interface numbering, plus the row's periodic neighbour indices.
struct RowWin {
    uint32_t wf, wc, r0, i0, pv, nv;
};

// From the LDS form; rf / rr point at the record's words xl / 32 and
// (xl + 1) / 32 pairs (f[2 k]), mr masks the bits below (xl + 1) % 32.
__device__ __forceinline__ RowWin row_window(const uint32_t *rw, const uint32_t *rr, const XRec &R, uint32_t sw,
                                             uint32_t mr) {
    RowWin o;
    o.wf = __builtin_amdgcn_alignbit(rw[2], rw[0], sw) & 7u;
    o.wc = __builtin_amdgcn_alignbit(rw[8], rw[6], sw) & 7u;
    o.r0 = rr[1] + uint32_t(__popc(rr[0] & mr));
    o.i0 = rr[7] + uint32_t(__popc(rr[6] & mr));
    o.pv = R.pv;
    o.nv = R.nv;
    return o;
}

// From a chunk record in registers (wavefronts that span too many units).
__device__ __forceinline__ RowWin row_window(const ChunkInfo &R, uint32_t xl, bool ledge, bool redge) {
    const uint32_t shr = ledge ? 0u : xl - 1u;
    const uint64_t below = (uint64_t(1) << xl) - 1u;
    const uint64_t fm = R.fluid, cm = R.cat;
    const uint32_t pv = R.prev, nv = R.next;
    uint32_t wf = uint32_t(ledge ? fm << 1 : fm >> shr) & 7u;
    uint32_t wc = uint32_t(ledge ? cm << 1 : cm >> shr) & 7u;
    wf |= ledge ? (pv >> 31) : 0u;
    wc |= ledge ? ((pv >> 30) & 1u) : 0u;
    wf = redge ? (wf & 3u) | ((nv >> 31) << 2) : wf;
    wc = redge ? (wc & 3u) | (((nv >> 30) & 1u) << 2) : wc;
    RowWin o;
    o.wf = wf;
    o.wc = wc;
    o.r0 = R.base + uint32_t(__popcll(fm & below));
    o.i0 = R.ibase + uint32_t(__popcll(cm & below));
    o.pv = pv & NB_IDX;
    o.nv = nv & NB_IDX;
    return o;
}

// Emission values of a wavefront's catalytic sources, read densely: the
// lanes list the interface indices of their catalytic sources in LDS,
// direction by direction at their rank among the lanes that have one (ballot
// and mbcnt), read the list 64 entries per pass, and take their values back
// in the same order.  A wavefront issues about one load per 64 sources
// instead of one per direction; the values are those of the direct reads.
// Wavefronts with more sources than the LDS list holds, or with idle
// lanes, read directly.
// gather: GATHER_BYTES of the wavefront's LDS, values first, then indices.
constexpr uint32_t GATHER_BYTES = 2048;
template <int ST>
__device__ __forceinline__ void gather_emission(const typename Store<ST>::S *__restrict__ emit, const uint32_t *kidx,
                                                uint32_t cat_bits, uint32_t *gather,
                                                typename Store<ST>::S (&re)[19]) {
    using S = typename Store<ST>::S;
    constexpr uint32_t CAP = GATHER_BYTES / (sizeof(S) + 4) / 64 * 64;  // 256 at FP32, 128 at FP64
    constexpr uint32_t PASSES = CAP / 64;
    S *vals = reinterpret_cast<S *>(gather);
    uint32_t *keys = gather + CAP * sizeof(S) / 4;
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t total = 0;  // the same in every lane
#pragma unroll
    for (int i = 1; i < 19; ++i)
        total += uint32_t(__popcll(__builtin_amdgcn_ballot_w64((cat_bits >> i) & 1u)));
    // the passes deal list entry t to lane t mod 64: a wavefront with idle
    // lanes (the last one of the domain) would leave their entries unread
    if (total > CAP || __builtin_amdgcn_read_exec() != ~0ull) {
#pragma unroll
        for (int i = 1; i < 19; ++i) {
            uint32_t v_b = kidx[(i - 1) * CTHREADS + threadIdx.x] * uint32_t(sizeof(S));
            opaque(v_b);
            re[i] = ld_at(emit, v_b);
        }
        return;
    }
    // the pull's LDS reads (the records this space held) before these writes
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    uint32_t at = 0;
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        const bool act = (cat_bits >> i) & 1u;
        const uint64_t b = __builtin_amdgcn_ballot_w64(act);
        if (act) keys[at + bits_below_lane(b)] = kidx[(i - 1) * CTHREADS + threadIdx.x];
        at += uint32_t(__popcll(b));
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    S v[PASSES];
#pragma unroll
    for (uint32_t q = 0; q < PASSES; ++q) {
        v[q] = S(0);
        if (q * 64u < total) {  // wave-uniform: only the passes the list needs
            const uint32_t t = q * 64u + lane;
            uint32_t v_b = (t < total ? keys[t] : 0u) * uint32_t(sizeof(S));
            opaque(v_b);
            v[q] = ld_at(emit, v_b);
        }
    }
#pragma unroll
    for (uint32_t q = 0; q < PASSES; ++q)
        if (q * 64u + lane < total) vals[q * 64u + lane] = v[q];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    at = 0;
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        const bool act = (cat_bits >> i) & 1u;
        const uint64_t b = __builtin_amdgcn_ballot_w64(act);
        re[i] = act ? vals[at + bits_below_lane(b)] : S(0);
        at += uint32_t(__popcll(b));
    }
}

// The same pull for the node-compact sweep: each lane is one gas node at
// (x, y, z) with storage index idx, lanes of a wave need not share a row.  For
// each of the nine source rows a lane reads the record of its own chunk in
// that row and takes a three-bit window (x - 1, x, x + 1) of its gas and
// catalytic masks; the chunk's edge bits and periodic neighbour ranks stand
// in where x -+ 1 leaves the chunk.  Same sources, same arithmetic and same
// decode as pull() above.
//
// Three phases keep a wave to two dependent memory round trips: all nine
// records are requested first; the windows and ranks are then worked out
// (interface indices go to kidx in LDS); then every population and emission
// load is issued before any is waited on.  Vector loads retire in order, so a
// record requested after population loads could not be waited on without
// waiting for those too.
//
// With the product flag in SP the product lattice is pulled alongside, from
// the same sources: no product at the inlet ghost, the outlet copy, and at a
// catalytic source E_P(k) (or, for reversal, p p_S^R times the reactant plus
// 1 - p_S^P times the product population that arrived along the reversed
// link: second sputtering equation).
// The sweeps where the emission gather is a choice: FP32 and FP64 storage,
// UNIFORM and WEIGHTED sputtering, no product lattice.
template <int ST, int SP>
constexpr bool gather_applies() {
    return SP >= 0 && sizeof(typename Store<ST>::S) >= 4 && (SP & SP_PRODUCT_FLAG) == 0 &&
           ((SP & 3) == SP_UNIFORM || (SP & 3) == SP_WEIGHTED);
}

template <int ST, int SP, bool GATHER_OK = true>
__device__ __forceinline__ void pull_c(const Geometry &g, const PhysK<typename Store<ST>::T> &ph, const Slots &in,
                                       const typename Store<ST>::S *__restrict__ emit, uint32_t idx, int x, int y,
                                       int z, typename Store<ST>::T (&hC)[19], typename Store<ST>::T (&hR)[19],
                                       uint32_t &cat_out, uint32_t *kidx, const ProdK<ST> &pk,
                                       typename Store<ST>::T (&hP)[19], const XRec *wrec, uint32_t wunit,
                                       uint32_t *gather) {
    using T = typename Store<ST>::T;
    using S = typename Store<ST>::S;
    using P = typename Store<ST>::P;
    constexpr uint32_t SB = sizeof(S), PB = 2 * SB;
    // source row class (cy, cz) of each group of directions in ORDER
    constexpr int CYS[9] = {0, 1, -1, 0, 0, 1, 1, -1, -1};
    constexpr int CZS[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
    const uint32_t nfp_b = in.stride;   // one slot, in bytes
    const bool reservoir = ph.species_x != XB_PERIODIC;  // inlet and outlet ghost planes
    // SP: the sputter mode (bits 0-1) and the INFLOW flag, fixed at compile
    // time for the sweeps, or -1 to read both from ph
    const int sputter = SP >= 0 ? (SP & 3) : ph.sputter;
    const bool inflow = SP >= 0 ? (SP & SP_INFLOW_FLAG) != 0 : ph.species_x == XB_INFLOW;
    const bool bounce = sputter == SP_BOUNCEBACK, uniform = sputter == SP_UNIFORM;
    const bool stoch = sputter == SP_STOCHASTIC;  // per-exit emission slots (already divided by w_i)
    const bool diffuse = SP >= 0 ? (SP & SP_DIFFUSE_FLAG) != 0 : ph.sigma != T(0);
    uint32_t solid_bits = 0;  // directions whose source is solid (the carrier reflects there)
    auto base = [&](int slot) { return in.p(slot); };
    const uint32_t own_e = node_elem(g, idx), own_b = own_e * PB;
    const uint32_t xl = uint32_t(x) & 63u, chunk = uint32_t(x) >> 6;
    const bool ledge = xl == 0u;                       // x - 1 lies in the previous chunk (or wraps)
    const bool redge = xl == 63u || x == g.nx - 1;     // x + 1 lies in the next chunk (or wraps)
    const bool first_x = x == 0, last_x = x == g.nx - 1;

    // phases 1 and 2: per source-row class, the lane's window bits and ranks
    // (RowWin), from the wavefront's LDS records (wrec, see wave_records) or,
    // where the wavefront spans too many units, from nine records of its own,
    // all requested before any is used.  Then the ranks of x - 1, x, x + 1
    // (rank - 1 and rank + 1 inside the row, the stored neighbours across the
    // periodic wrap), the catalytic sources, and their interface indices to
    // kidx.
    uint32_t wins = 0;  // three gas bits (x - 1, x, x + 1) per class
    uint32_t rk[9][3];  // storage index of x - 1, x, x + 1 in each source row (where gas)
    uint32_t cat_bits = 0;
    // catalytic sources need a gas-free interface voxel; the reservoir planes
    // take the place of the wrapped x - 1 at x = 0 and x + 1 at x = nx - 1
    const uint32_t cat_ok = 7u & ~((reservoir && first_x) ? 1u : 0u) & ~((reservoir && last_x) ? 4u : 0u);
    auto take = [&](const int cls, const RowWin &W) {
        const int cy = CYS[cls], cz = CZS[cls];
        rk[cls][1] = W.r0;
        rk[cls][0] = first_x ? W.pv : W.r0 - 1u;
        rk[cls][2] = last_x ? W.nv : W.r0 + ((W.wf >> 1) & 1u);
        const uint32_t im = first_x ? W.pv : W.i0 - 1u;
        const uint32_t ip = last_x ? W.nv : W.i0 + ((W.wc >> 1) & 1u);
        const uint32_t cw = W.wc & ~W.wf & cat_ok;
        wins |= W.wf << (3 * cls);
#pragma unroll
        for (int k = 0; k < 18; ++k) {
            const int i = ORDER[k];
            if (CY[i] != cy || CZ[i] != cz) continue;
            const int cx = CX[i];
            const int bit = 1 - cx;
            const uint32_t m = uint32_t(int32_t(cw << (31 - bit)) >> 31);  // all ones where catalytic
            const uint32_t irank = cx == 0 ? W.i0 : (cx == 1 ? im : ip);
            kidx[(i - 1) * CTHREADS + threadIdx.x] = m & irank;
            cat_bits |= m & (1u << i);
        }
    };
    if (wrec) {
        const XRec *R0 = wrec + wunit * 9u;
        const uint32_t sw = xl & 31u, kw = xl >> 5, kr = (xl + 1u) >> 5;
        const uint32_t mr = (1u << ((xl + 1u) & 31u)) - 1u;
        const uint32_t *rw = R0[0].f + 2u * kw, *rr = R0[0].f + 2u * kr;
        constexpr uint32_t XW = sizeof(XRec) / 4u;
#pragma unroll
        for (int cls = 0; cls < 9; ++cls) take(cls, row_window(rw + cls * XW, rr + cls * XW, R0[cls], sw, mr));
    } else {
        ChunkInfo rec[9];
#pragma unroll
        for (int cls = 0; cls < 9; ++cls) {
            int ys = y - CYS[cls], zs = z - CZS[cls];
            ys = ys < 0 ? ys + g.ny : (ys >= g.ny ? ys - g.ny : ys);
            zs = zs < 0 ? zs + g.nz : (zs >= g.nz ? zs - g.nz : zs);
            const uint32_t rown = uint32_t(zs) * uint32_t(g.ny) + uint32_t(ys);
            const LBM_GLOBAL ChunkInfo &src = glb(g.chunks)[rown * uint32_t(g.W) + chunk];
            rec[cls].fluid = src.fluid;
            rec[cls].cat = src.cat;
            rec[cls].base = src.base;
            rec[cls].ibase = src.ibase;
            rec[cls].prev = src.prev;
            rec[cls].next = src.next;
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int cls = 0; cls < 9; ++cls) take(cls, row_window(rec[cls], xl, ledge, redge));
    }

    // phase 3: every population and emission load.  One load per direction
    // gives both lattices (same gas source, or both bounced back); the
    // reactant differs only at catalytic sources (emission), at the inlet
    // plane (the reservoir value) and at the outlet plane (a copy of plane
    // nx - 1, loaded only by wavefronts that hold an outlet lane).
    P pc[19];
    S re[19], ro[19];
    constexpr bool PROD = SP >= 0 && (SP & SP_PRODUCT_FLAG) != 0;
    // Emission reads gathered densely (see gather_emission) where the
    // launch asks for it (GATHER_OK, the emission tunable) and the gather
    // applies (gather_applies: FP32 and FP64 storage, the UNIFORM and
    // WEIGHTED modes with one emission value per interface node, no product
    // lattice).  It trades vector-memory loads for VALU work; which wins
    // depends on the workload (630 against 634 us for the 256^3 sweep, 2216
    // against 2166 us for the 64-sample batched sweep), so it is measured.
    constexpr bool GATHER = GATHER_OK && gather_applies<ST, SP>();
    S pp[PROD ? 19 : 1], pe[PROD ? 19 : 1], po[PROD ? 19 : 1];
    const uint32_t nfpp_b = pk.in.stride, ownp_b = own_e * SB;  // product buffer: one population per element
    pc[0] = ld_pop<ST>(base(dslot(0)), own_b);
    if constexpr (PROD) pp[0] = ld_at(static_cast<const S *>(pk.in.p(dslot(0))), ownp_b);
    const bool any_outlet = reservoir && __builtin_amdgcn_ballot_w64(last_x) != 0u;
#pragma unroll
    for (int cls = 0; cls < 9; ++cls) {
        const int cy = CYS[cls], cz = CZS[cls];
        const uint32_t wf = (wins >> (3 * cls)) & 7u;
#pragma unroll
        for (int k = 0; k < 18; ++k) {
            const int i = ORDER[k];
            if (CY[i] != cy || CZ[i] != cz) continue;
            const int cx = CX[i];
            const uint32_t bit = uint32_t(1 - cx);
            const bool F = (wf >> bit) & 1u;
            const uint32_t fmask = uint32_t(int32_t(wf << (31 - bit)) >> 31);  // all ones where the source is gas
            const uint32_t half = dslot(i) < dslot(opp(i)) ? 0u : nfp_b;
            const uint32_t bb_b = own_b + (nfp_b - half);
            const uint32_t rke = node_elem(g, rk[cls][bit]);
            const uint32_t pull_b = rke * PB + half;
            uint32_t c_b = (pull_b & fmask) | (bb_b & ~fmask);
            solid_bits |= ~fmask & (1u << i);
            opaque(c_b);
            pc[i] = ld_pop<ST>(base(pair_slot(i)), c_b);
            if constexpr (!GATHER) {
                uint32_t v_b = bounce ? 0u
                                      : (stoch ? uint32_t(i - 1) * g.niface + kidx[(i - 1) * CTHREADS + threadIdx.x]
                                               : kidx[(i - 1) * CTHREADS + threadIdx.x]) * SB;
                opaque(v_b);
                re[i] = ld_at(emit, v_b);
            }
            ro[i] = S(0);
            if (cx == -1 && any_outlet) {
                const bool F0 = (wf >> 1) & 1u;
                uint32_t o_b = (last_x && F0 ? node_elem(g, rk[cls][1]) * PB + half : bb_b) + SB;
                opaque(o_b);
                ro[i] = ld_at(static_cast<const S *>(base(pair_slot(i))), o_b);
            }
            if constexpr (PROD) {
                const uint32_t halfp = dslot(i) < dslot(opp(i)) ? 0u : nfpp_b;
                const uint32_t bbp_b = ownp_b + (nfpp_b - halfp);
                const S *pbase = static_cast<const S *>(pk.in.p(pair_slot(i)));
                uint32_t p_b = F ? rke * SB + halfp : bbp_b;
                opaque(p_b);
                pp[i] = ld_at(pbase, p_b);
                uint32_t e_b = bounce ? 0u : kidx[(i - 1) * CTHREADS + threadIdx.x] * SB;
                opaque(e_b);
                pe[i] = ld_at(pk.emit, e_b);
                po[i] = S(0);
                if (cx == -1 && any_outlet) {
                    const bool F0 = (wf >> 1) & 1u;
                    uint32_t o_b = last_x && F0 ? node_elem(g, rk[cls][1]) * SB + halfp : bbp_b;
                    opaque(o_b);
                    po[i] = ld_at(pbase, o_b);
                }
            }
        }
    }
    if constexpr (GATHER) gather_emission<ST>(emit, kidx, cat_bits, gather, re);
    __builtin_amdgcn_sched_barrier(0);
    const T h_in = Store<ST>::cv(Store<ST>::enc(ph.h_inlet));
    const bool inlet = reservoir && first_x, outlet = reservoir && last_x;
    hC[0] = Store<ST>::cv(pc[0].x);
    hR[0] = Store<ST>::cv(pc[0].y);
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        hC[i] = Store<ST>::cv(pc[i].x);
        T v = Store<ST>::cv(pc[i].y);
        if (CX[i] == 1) v = inlet ? h_in : v;
        if (CX[i] == -1) v = outlet ? Store<ST>::cv(ro[i]) : v;
        const T ev = Store<ST>::cv(re[i]);
        const T v_cat = bounce ? ph.keep * (v + ph.cref) - ph.cref : (uniform ? ev * inv_wgt<T>(i) : ev) - ph.cref;
        if constexpr (PROD) {
            T q = Store<ST>::cv(pp[i]);
            if (CX[i] == 1) q = inlet ? T(0) : q;
            if (CX[i] == -1) q = outlet ? Store<ST>::cv(po[i]) : q;
            const T epv = Store<ST>::cv(pe[i]);
            const T q_cat = bounce ? ph.a_r * (v + ph.cref) + ph.a_p * q : (uniform ? epv * inv_wgt<T>(i) : epv);
            hP[i] = ((cat_bits >> i) & 1u) ? q_cat : q;
        }
        hR[i] = ((cat_bits >> i) & 1u) ? v_cat : v;
    }
    if constexpr (PROD) hP[0] = Store<ST>::cv(pp[0]);
    // the reference flow (none with FP32 storage, whose sweep is register bound)
    const bool shifted = ST != ST_F32 && ph.us3 != T(0);
    if constexpr (ST != ST_F32)
        if (shifted) bounced_half_shift(ph, solid_bits, hC);
    if (diffuse && solid_bits != 0u) diffuse_wall(ph.sigma, solid_bits, hC);
    if constexpr (ST != ST_F32)
        if (shifted) bounced_half_shift(ph, solid_bits, hC);
    if (inflow && __builtin_amdgcn_ballot_w64(first_x) != 0u && first_x) inflow_ghost(ph, hC, hR);
    cat_out = cat_bits;
}

// Moments of both lattices and the equilibrium velocity.
template <typename T>
struct Mom {
    T dc, rc, dr, rr;  // density deviations and densities
    T ux, uy, uz;
};

template <typename T>
__device__ __forceinline__ void weighted_moments(const T (&h)[19], T &d, T &jx, T &jy, T &jz) {
    // sum_i w_i h_i and sum_i w_i c_i h_i, grouped by weight class
    T axis = 0, diag = 0, ax = 0, ay = 0, az = 0, gx = 0, gy = 0, gz = 0;
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        const bool is_axis = CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i] == 1;
        T &sum = is_axis ? axis : diag;
        sum += h[i];
        T &mx = is_axis ? ax : gx;
        T &my = is_axis ? ay : gy;
        T &mz = is_axis ? az : gz;
        if (CX[i] == 1) mx += h[i];
        if (CX[i] == -1) mx -= h[i];
        if (CY[i] == 1) my += h[i];
        if (CY[i] == -1) my -= h[i];
        if (CZ[i] == 1) mz += h[i];
        if (CZ[i] == -1) mz -= h[i];
    }
    d = wgt<T>(0) * h[0] + wgt<T>(1) * axis + wgt<T>(4) * diag;
    jx = wgt<T>(1) * ax + wgt<T>(4) * gx;
    jy = wgt<T>(1) * ay + wgt<T>(4) * gy;
    jz = wgt<T>(1) * az + wgt<T>(4) * gz;
}

template <typename T>
__device__ __forceinline__ Mom<T> moments(const PhysK<T> &ph, const T (&hC)[19], const T (&hR)[19]) {
    Mom<T> m;
    T jx, jy, jz;
    weighted_moments(hC, m.dc, jx, jy, jz);
    m.rc = ph.rref + m.dc;
    if (ph.coupling == CP_BARYCENTRIC) {
        T rx, ry, rz;
        weighted_moments(hR, m.dr, rx, ry, rz);
        m.rr = ph.cref + m.dr;
        const T inv = T(1) / (m.rc + m.rr);
        m.ux = (jx + ph.usx + rx + T(0.5) * ph.fx) * inv;
        m.uy = (jy + ry + T(0.5) * ph.fy) * inv;
        m.uz = (jz + rz + T(0.5) * ph.fz) * inv;
    } else {
        T axis = 0, diag = 0;
#pragma unroll
        for (int i = 1; i < 19; ++i) {
            if (CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i] == 1)
                axis += hR[i];
            else
                diag += hR[i];
        }
        m.dr = wgt<T>(0) * hR[0] + wgt<T>(1) * axis + wgt<T>(4) * diag;
        m.rr = ph.cref + m.dr;
        const T inv = T(1) / m.rc;
        // jx is the shifted form's x-moment: the true one less usx
        m.ux = (jx + ph.usx + T(0.5) * ph.fx) * inv;
        m.uy = (jy + T(0.5) * ph.fy) * inv;
        m.uz = (jz + T(0.5) * ph.fz) * inv;
    }
    return m;
}

// BGK collision in normalised form: h* = h - omega (h - heq) (+ Guo / w_i on
// the carrier), heq_i = (rho - rho_ref) + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u);
// the carrier's h and heq both in the shifted form (less 3 c_ix U).
// Directions are taken in opposite pairs (c.u and c.F change sign), which
// shares most of the arithmetic between the two.
template <typename T>
__device__ __forceinline__ void collide(const PhysK<T> &ph, const Mom<T> &m, T (&hC)[19], T (&hR)[19]) {
    const T uu = m.ux * m.ux + m.uy * m.uy + m.uz * m.uz;
    const T uf = m.ux * ph.fx + m.uy * ph.fy + m.uz * ph.fz;
    const T base_c = m.dc - T(1.5) * m.rc * uu, base_r = m.dr - T(1.5) * m.rr * uu;
    const T guo3 = T(3) * ph.guo, guo9 = T(9) * ph.guo;
    // h - omega (h - heq) keeps the small non-equilibrium part exact
    hC[0] = hC[0] - ph.om_c * (hC[0] - base_c) - guo3 * uf;
    hR[0] = hR[0] - ph.om_r * (hR[0] - base_r);
#pragma unroll
    for (int i = 1; i <= 9; ++i) {
        const int j = opp(i);
        const T cu = T(CX[i]) * m.ux + T(CY[i]) * m.uy + T(CZ[i]) * m.uz;
        const T cf = T(CX[i]) * ph.fx + T(CY[i]) * ph.fy + T(CZ[i]) * ph.fz;  // wave-uniform
        const T q = T(4.5) * cu * cu, l = T(3) * cu;
        // the carrier's linear equilibrium term 3 rho c.u in its shifted form
        // (less 3 c_x U)
        const T tc = base_c + m.rc * q, sc = m.rc * l - T(CX[i]) * ph.us3;
        const T tr = base_r + m.rr * q, sr = m.rr * l;
        const T a = guo9 * cu * cf - guo3 * uf, b = guo3 * cf;  // Guo term: a + b (i), a - b (opp)
        hC[i] = hC[i] - ph.om_c * (hC[i] - (tc + sc)) + (a + b);
        hC[j] = hC[j] - ph.om_c * (hC[j] - (tc - sc)) + (a - b);
        hR[i] = hR[i] - ph.om_r * (hR[i] - (tr + sr));
        hR[j] = hR[j] - ph.om_r * (hR[j] - (tr - sr));
    }
}

// ------------------------------------------------------------ kernels --

// Reactant leaving through x = -1 (own post-collision populations of x = 0
// along c_x = -1) or x = nx (of x = nx - 1 along c_x = +1), and the influx
// pulled at x = 0.  Out of line: it runs on two lanes per x-row and would
// otherwise raise the register budget of the whole sweep.
struct InOut {
    double in, out;
};

// Add this lane's post-collision reactant populations that head into
// interface nodes (the reversed catalytic-source directions) to In(k) of
// their targets, as fixed-point integers; kidx holds each direction's target.
// hR holds the values as stored (the sweeps write the rounded 16-bit values
// back before calling), so In(k) counts exactly the mass that left.
template <int ST, uint32_t KS = 256>
__device__ __forceinline__ void accumulate_in(unsigned long long *inacc, const uint32_t *kidx, uint32_t cat_bits,
                                              const PhysK<typename Store<ST>::T> &ph,
                                              const typename Store<ST>::T (&hR)[19],
                                              typename Store<ST>::T cref) {
    using T = typename Store<ST>::T;
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        if ((cat_bits >> i) & 1u) {
            const int j = opp(i);  // the link direction as seen from the interface node
            const T stored = hR[j];  // the value as stored (the caller passes stored values)
            (void)__hip_atomic_fetch_add(&glb(inacc)[kidx[(i - 1) * KS + threadIdx.x]],
                                         in_term<T>(wgt<T>(j), stored, cref, ph.in_scale), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// STOCHASTIC: the same terms, each added to the In slot of the exit its draw
// picks.  Slots receive a random number of terms, so the terms are plain
// two's-complement integers (the fixed-point pattern minus MAGIC_BITS) and
// the reader subtracts nothing.
//
// The draws are made densely: each wavefront queues its arrivals (term,
// interface node, link code) in LDS, direction by direction, and draws the
// exits of 64 queued arrivals per pass, so a wavefront runs the generator
// about once instead of once per direction in which any of its lanes has a
// catalytic source.  Integer sums do not depend on the order, so the slots
// hold the same values.
struct QueuedArrival {
    unsigned long long term;
    uint32_t k, code;
};
constexpr uint32_t ARRIVAL_QUEUE = 128;  // per wavefront: < 64 waiting + up to one per live lane added

// The entries are dealt over the lanes active here (the calling sweep runs
// only its gas-node lanes), by their rank among them.
__device__ __forceinline__ void draw_queued(const QueuedArrival *q, uint32_t n, const uint32_t *ivox,
                                         const uint32_t *imask, unsigned long long *inacc, uint32_t niface,
                                         uint32_t step, uint32_t seed_lo, uint32_t seed_hi) {
    const uint64_t live = __builtin_amdgcn_read_exec();
    const uint32_t rank = __builtin_amdgcn_mbcnt_hi(uint32_t(live >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(live), 0u));
    const uint32_t lanes = uint32_t(__popcll(live));
    for (uint32_t t = rank; t < n; t += lanes) {
        const QueuedArrival a = q[t];
        const int e = random_exit(step, seed_lo, seed_hi, glb(ivox)[a.k], glb(imask)[a.k], a.code);
        (void)__hip_atomic_fetch_add(&glb(inacc)[uint64_t(uint32_t(e - 1)) * niface + a.k], a.term,
                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// The direct form (a draw in place per direction), for the chunk sweep,
// whose register budget the queue would exceed.
template <int ST>
__device__ __forceinline__ void accumulate_in_random_direct(const Geometry &g, unsigned long long *inacc,
                                                            const uint32_t *kidx, uint32_t cat_bits,
                                                            const PhysK<typename Store<ST>::T> &ph,
                                                            const typename Store<ST>::T (&hR)[19]) {
    using T = typename Store<ST>::T;
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        if ((cat_bits >> i) & 1u) {
            const int j = opp(i);  // the link direction as seen from the interface node
            const uint32_t k = kidx[(i - 1) * 256 + threadIdx.x];
            const int e = random_exit(ph.step_ctr, ph.seed_lo, ph.seed_hi, glb(g.ivox)[k], glb(g.imask)[k],
                                      uint32_t(vcode(j)));
            const T stored = hR[j];  // as stored
            const unsigned long long term = in_term<T>(wgt<T>(j), stored, ph.cref, ph.in_scale) - MAGIC_BITS;
            (void)__hip_atomic_fetch_add(&glb(inacc)[uint64_t(uint32_t(e - 1)) * g.niface + k], term,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <int ST>
__device__ __forceinline__ void accumulate_in_random(const Geometry &g, unsigned long long *inacc,
                                                     const uint32_t *kidx, uint32_t cat_bits,
                                                     const PhysK<typename Store<ST>::T> &ph,
                                                     const typename Store<ST>::T (&hR)[19], QueuedArrival *q) {
    using T = typename Store<ST>::T;
    uint32_t qn = 0;  // the same in every lane of the wavefront
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        const bool act = (cat_bits >> i) & 1u;
        const uint64_t bal = __builtin_amdgcn_ballot_w64(act);
        if (bal == 0u) continue;
        if (act) {
            const int j = opp(i);  // the link direction as seen from the interface node
            const T stored = hR[j];  // as stored
            QueuedArrival a;
            a.term = in_term<T>(wgt<T>(j), stored, ph.cref, ph.in_scale) - MAGIC_BITS;
            a.k = kidx[(i - 1) * CTHREADS + threadIdx.x];
            a.code = uint32_t(vcode(j));
            const uint32_t below = __builtin_amdgcn_mbcnt_hi(uint32_t(bal >> 32),
                                                             __builtin_amdgcn_mbcnt_lo(uint32_t(bal), 0u));
            q[qn + below] = a;
        }
        qn += uint32_t(__popcll(bal));
        if (qn >= 64u) {
            // the wavefront's queue writes before its reads, and its reads
            // before the next writes (LDS accesses of one wavefront)
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            draw_queued(q, qn, g.ivox, g.imask, inacc, g.niface, ph.step_ctr, ph.seed_lo, ph.seed_hi);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            qn = 0;
        }
    }
    if (qn > 0u) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        draw_queued(q, qn, g.ivox, g.imask, inacc, g.niface, ph.step_ctr, ph.seed_lo, ph.seed_hi);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
}

// The same terms as accumulate_in, queued densely in LDS direction by
// direction and added 64 per pass: a wavefront issues about one atomic
// instruction per 64 arrivals instead of one per direction in which any of
// its lanes has a catalytic source.  The sums are integers, so In(k) holds the
// same bits as with accumulate_in.
__device__ __forceinline__ void add_queued(const QueuedArrival *q, uint32_t n, unsigned long long *inacc) {
    const uint64_t live = __builtin_amdgcn_read_exec();
    const uint32_t rank = __builtin_amdgcn_mbcnt_hi(uint32_t(live >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(live), 0u));
    const uint32_t lanes = uint32_t(__popcll(live));
    for (uint32_t t = rank; t < n; t += lanes) {
        const QueuedArrival a = q[t];
        (void)__hip_atomic_fetch_add(&glb(inacc)[a.k], a.term, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <int ST>
__device__ __forceinline__ void accumulate_in_queued(unsigned long long *inacc, const uint32_t *kidx,
                                                     uint32_t cat_bits, const PhysK<typename Store<ST>::T> &ph,
                                                     const typename Store<ST>::T (&hR)[19],
                                                     typename Store<ST>::T cref, QueuedArrival *q) {
    using T = typename Store<ST>::T;
    uint32_t qn = 0;  // the same in every lane of the wavefront
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        const bool act = (cat_bits >> i) & 1u;
        const uint64_t bal = __builtin_amdgcn_ballot_w64(act);
        if (bal == 0u) continue;
        if (act) {
            const int j = opp(i);  // the link direction as seen from the interface node
            QueuedArrival a;
            a.term = in_term<T>(wgt<T>(j), hR[j], cref, ph.in_scale);
            a.k = kidx[(i - 1) * CTHREADS + threadIdx.x];
            a.code = 0u;
            const uint32_t below = __builtin_amdgcn_mbcnt_hi(uint32_t(bal >> 32),
                                                             __builtin_amdgcn_mbcnt_lo(uint32_t(bal), 0u));
            q[qn + below] = a;
        }
        qn += uint32_t(__popcll(bal));
        if (qn >= 64u) {
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            add_queued(q, qn, inacc);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            qn = 0;
        }
    }
    if (qn > 0u) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        add_queued(q, qn, inacc);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
}

// The compact sweep's choice: queued at FP32 and FP64 storage, whose sweeps
// are bound by vector-memory instructions (measured at 256^3 FP32: 648 ->
// 636 us); direct at 16 bits, where the queue's extra VALU and LDS work costs
// more than the instructions it saves (455 -> 468 us).
template <int ST>
__device__ __forceinline__ void accumulate_in_c(unsigned long long *inacc, const uint32_t *kidx, uint32_t cat_bits,
                                                const PhysK<typename Store<ST>::T> &ph,
                                                const typename Store<ST>::T (&hR)[19], typename Store<ST>::T cref,
                                                QueuedArrival *q) {
    if constexpr (sizeof(typename Store<ST>::S) == 2)
        accumulate_in<ST, CTHREADS>(inacc, kidx, cat_bits, ph, hR, cref);
    else
        accumulate_in_queued<ST>(inacc, kidx, cat_bits, ph, hR, cref, q);
}

template <int ST>
__device__ __noinline__ InOut boundary_tally(typename Store<ST>::T c_ref, double c_in, const char *pop,
                                             uint32_t stride, uint32_t elem, bool first_x, bool last_x) {
    using T = typename Store<ST>::T;
    using S = typename Store<ST>::S;
    // the node's own reactant population of direction i (elem: its element index)
    auto own = [&](int i) {
        return Store<ST>::ld(reinterpret_cast<const S *>(pop + uint64_t(dslot(i)) * stride) + 2 * uint64_t(elem) + 1);
    };
    double fin = 0.0, fout = 0.0;
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        if (CX[i] == 1) {
            if (first_x) fin += double(wgt<T>(i)) * c_in;
            if (last_x) fout += double(wgt<T>(i) * (own(i) + c_ref));
        }
        if (CX[i] == -1 && first_x) fout += double(wgt<T>(i) * (own(i) + c_ref));
    }
    return InOut{fin, fout};
}

// Product leaving through the x-faces: out_in, its own post-collision
// populations at x = 0 along c_x = -1; out_out, those at x = nx - 1 along
// c_x = +1 (what the outlet ghost returned is subtracted by the caller).
template <int ST>
__device__ __noinline__ InOut product_tally(const char *pop, uint32_t stride, uint32_t elem, bool first_x,
                                            bool last_x) {
    using T = typename Store<ST>::T;
    using S = typename Store<ST>::S;
    auto own = [&](int i) {
        return Store<ST>::ld(reinterpret_cast<const S *>(pop + uint64_t(dslot(i)) * stride) + elem);
    };
    double oin = 0.0, oout = 0.0;
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        if (CX[i] == 1 && last_x) oout += double(wgt<T>(i) * own(i));
        if (CX[i] == -1 && first_x) oin += double(wgt<T>(i) * own(i));
    }
    return InOut{oin, oout};
}

// BGK collision of the product lattice with the velocity of the carrier
// (stored unshifted: h_eq = rho (1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u.u)).
template <typename T>
__device__ __forceinline__ void collide_product(const PhysK<T> &ph, const Mom<T> &m, T rp, T (&hP)[19]) {
    const T uu = m.ux * m.ux + m.uy * m.uy + m.uz * m.uz;
    const T base = rp - T(1.5) * rp * uu;
    hP[0] = hP[0] - ph.om_r * (hP[0] - base);
#pragma unroll
    for (int i = 1; i <= 9; ++i) {
        const int j = opp(i);
        const T cu = T(CX[i]) * m.ux + T(CY[i]) * m.uy + T(CZ[i]) * m.uz;
        const T t = base + rp * (T(4.5) * cu * cu), sl = rp * (T(3) * cu);
        hP[i] = hP[i] - ph.om_r * (hP[i] - (t + sl));
        hP[j] = hP[j] - ph.om_r * (hP[j] - (t - sl));
    }
}

// One block of the fused sweep: logical block `block` of the sample described
// by g / ph, reading `in` and writing `out`; its four partial sums go to row
// `block` of `part`.
template <int ST, int SP>
__device__ __forceinline__ void sweep_block(const Geometry &g, const PhysK<typename Store<ST>::T> &ph, const Slots &in,
                                            const OutSlots &out, const typename Store<ST>::S *__restrict__ emit,
                                            double *__restrict__ part, uint32_t block) {
    using T = typename Store<ST>::T;
    const WaveUnit u = locate(g, block);
    __shared__ uint32_t kidx[18 * 256];
    // per-block partials: carrier mass, reactant mass, influx, outflux
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (u.active) {
        T hC[19], hR[19];
        uint32_t cat_bits;
        pull<ST, SP>(g, ph, in, emit, u, hC, hR, cat_bits, kidx);
        const Mom<T> m = moments(ph, hC, hR);
        acc[0] = double(m.rc);
        acc[1] = double(m.rr);
        // Reactant crossing the reservoir planes in this streaming: what the
        // outlet ghost returned to x = nx - 1 (pulled along c_x = -1) counts
        // against what left there (below).
        const bool reservoir = ph.species_x != XB_PERIODIC;  // inlet and outlet ghost planes
        const bool inflow = (SP & SP_INFLOW_FLAG) != 0;
        const bool first_x = u.x == 0, last_x = u.x == g.nx - 1;
        if (reservoir && last_x) {
#pragma unroll
            for (int i = 1; i < 19; ++i)
                if (CX[i] == -1) acc[3] -= double(wgt<T>(i) * (hR[i] + ph.cref));
        }
        if (inflow && first_x) {  // what the moving inlet ghost supplied
#pragma unroll
            for (int i = 1; i < 19; ++i)
                if (CX[i] == 1) acc[2] += double(wgt<T>(i) * (hR[i] + ph.cref));
        }
        collide(ph, m, hC, hR);
        using P = typename Store<ST>::P;
        uint32_t own_b = node_elem(g, u.idx) * uint32_t(sizeof(P));
        const lbmfx::RoundWords rw = lbmfx::round_words(ph.sr != 0u, ph.sr_key, u.idx);
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            // opaque per store: keeps each store in the scalar-base form instead
            // of a shared 64-bit vector address plus per-store 64-bit adds
            opaque(own_b);
            const P v = Store<ST>::enc2(hC[i], hR[i], rw.at(2 * i), rw.at(2 * i + 1));
            st_at(static_cast<P *>(out.p(dslot(i))), own_b, v);
            if constexpr (Store<ST>::ROUNDS) hR[i] = Store<ST>::cv(v.y);
        }
        // In(k) of the next step's interface: what leaves towards interface nodes
        if (__builtin_amdgcn_ballot_w64(cat_bits != 0u)) {
            if constexpr ((SP & 3) == SP_STOCHASTIC)
                accumulate_in_random_direct<ST>(g, g.inacc, kidx, cat_bits, ph, hR);
            else
                accumulate_in<ST>(g.inacc, kidx, cat_bits, ph, hR, ph.cref);
        }
        if (reservoir && (first_x || last_x)) {
            const InOut f = boundary_tally<ST>(ph.cref, inflow ? 0.0 : ph.c_in, in.base, in.stride, node_elem(g, u.idx),
                                               first_x,
                                               last_x);
            acc[2] += f.in;
            acc[3] += f.out;
        }
    }
    block_sum<4>(acc, part + int64_t(block) * 4);
}

// One block (one wavefront) of the node-compact sweep: wave slot `block`
// takes the 64 gas nodes of wave worder[slot] (storage indices 64 w .. 64 w +
// 63).
template <int ST, int SP, bool GATHER_OK = true>
__device__ __forceinline__ void sweep_block_c(const Geometry &g, const PhysK<typename Store<ST>::T> &ph,
                                              const Slots &in, const OutSlots &out,
                                              const typename Store<ST>::S *__restrict__ emit,
                                              double *__restrict__ part, uint32_t block, const ProdK<ST> &pk) {
    using T = typename Store<ST>::T;
    constexpr bool PROD = (SP & SP_PRODUCT_FLAG) != 0;
    double accp[3] = {0.0, 0.0, 0.0};  // product mass, out through the inlet face, out through the outlet face
    const uint32_t slot = block;
    const bool wvalid = slot < g.nwaves;
    const uint32_t w = glb(g.worder)[wvalid ? slot : 0u];
    const uint32_t idx = w * 64u + (threadIdx.x & 63u);
    const bool active = wvalid && int64_t(idx) < g.nfluid;
    __shared__ uint32_t kidx[18 * CTHREADS];
    // the records are dead once the pull has read them; the arrival queue
    // of the In(k) sums reuses their LDS
    __shared__ union {
        WaveRecords wrec;
        QueuedArrival queue[ARRIVAL_QUEUE];
    } lds;
    static_assert(sizeof(lds) >= GATHER_BYTES, "the emission gather list lives in the records' LDS");
    WaveRecords &wrec = lds.wrec;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    uint32_t wunit = 0, p = 0;
    const bool coop = wvalid && wave_records(g, w, idx, active, wrec, wunit, p);
    if (!coop && active) p = glb(g.pos)[idx];
    const int x = int(p & 0xfffu), y = int((p >> 12) & 0x3ffu), z = int(p >> 22);
    if (active) {
        T hC[19], hR[19], hP[19];  // hP: product lattice (unused without it)
        uint32_t cat_bits;
        pull_c<ST, SP, GATHER_OK>(g, ph, in, emit, idx, x, y, z, hC, hR, cat_bits, kidx, pk, hP,
                       coop ? wrec.rec : nullptr, wunit, reinterpret_cast<uint32_t *>(lds.queue));
        const Mom<T> m = moments(ph, hC, hR);
        acc[0] = double(m.rc);
        acc[1] = double(m.rr);
        const bool reservoir = ph.species_x != XB_PERIODIC;  // inlet and outlet ghost planes
        const bool inflow = (SP & SP_INFLOW_FLAG) != 0;
        const bool first_x = x == 0, last_x = x == g.nx - 1;
        if (reservoir && last_x) {
#pragma unroll
            for (int i = 1; i < 19; ++i)
                if (CX[i] == -1) acc[3] -= double(wgt<T>(i) * (hR[i] + ph.cref));
        }
        T rp = T(0);
        if constexpr (PROD) {
            T dpx, dpy, dpz;
            weighted_moments(hP, rp, dpx, dpy, dpz);
            accp[0] = double(rp);
            if (reservoir && last_x) {
#pragma unroll
                for (int i = 1; i < 19; ++i)
                    if (CX[i] == -1) accp[2] -= double(wgt<T>(i) * hP[i]);
            }
        }
        if (inflow && first_x) {  // what the moving inlet ghost supplied
#pragma unroll
            for (int i = 1; i < 19; ++i)
                if (CX[i] == 1) acc[2] += double(wgt<T>(i) * (hR[i] + ph.cref));
        }
        collide(ph, m, hC, hR);
        using P = typename Store<ST>::P;
        const uint32_t own_e = node_elem(g, idx);
        uint32_t own_b = own_e * uint32_t(sizeof(P));
        // the rounding words of this node (16-bit storage; nearest unless
        // stochastic rounding is on): 2i, 2i + 1 for the pair of direction i,
        // 38 + i for the product
        const lbmfx::RoundWords rw = lbmfx::round_words(ph.sr != 0u, ph.sr_key, idx);
        auto store_pairs = [&](const bool stochastic) {
#pragma unroll
            for (int i = 0; i < 19; ++i) {
                opaque(own_b);
                // rounding to nearest uses one constant word: no per-word arithmetic
                const uint32_t wc = stochastic ? rw.at(2 * i) : lbmfx::ROUND_NEAREST_BITS;
                const uint32_t wr = stochastic ? rw.at(2 * i + 1) : lbmfx::ROUND_NEAREST_BITS;
                const P v = Store<ST>::enc2(hC[i], hR[i], wc, wr);
                st_stream(static_cast<P *>(out.p(dslot(i))), own_b, v);
                if constexpr (Store<ST>::ROUNDS) hR[i] = Store<ST>::cv(v.y);
            }
        };
        if constexpr (Store<ST>::ROUNDS) {
            if (ph.sr != 0u)
                store_pairs(true);
            else
                store_pairs(false);
        } else {
            store_pairs(false);
        }
        if constexpr (PROD) {
            using S = typename Store<ST>::S;
            collide_product(ph, m, rp, hP);
            uint32_t ownp_b = own_e * uint32_t(sizeof(S));
#pragma unroll
            for (int i = 0; i < 19; ++i) {
                opaque(ownp_b);
                const S v = Store<ST>::enc1(hP[i], rw.at(38 + i));
                st_stream(static_cast<S *>(pk.out.p(dslot(i))), ownp_b, v);
                if constexpr (Store<ST>::ROUNDS) hP[i] = Store<ST>::cv(v);
            }
            if (__builtin_amdgcn_ballot_w64(cat_bits != 0u))
                accumulate_in_c<ST>(pk.inacc, kidx, cat_bits, ph, hP, T(0), lds.queue);
            if (reservoir && (first_x || last_x)) {
                const InOut f = product_tally<ST>(pk.in.base, pk.in.stride, node_elem(g, idx), first_x, last_x);
                accp[1] += f.in;
                accp[2] += f.out;
            }
        }
        if (__builtin_amdgcn_ballot_w64(cat_bits != 0u)) {
            if constexpr ((SP & 3) == SP_STOCHASTIC)
                accumulate_in_random<ST>(g, g.inacc, kidx, cat_bits, ph, hR, lds.queue);
            else
                accumulate_in_c<ST>(g.inacc, kidx, cat_bits, ph, hR, ph.cref, lds.queue);
        }
        if (reservoir && (first_x || last_x)) {
            const InOut f = boundary_tally<ST>(ph.cref, inflow ? 0.0 : ph.c_in, in.base, in.stride, node_elem(g, idx),
                                               first_x,
                                               last_x);
            acc[2] += f.in;
            acc[3] += f.out;
        }
    }
    wave_partials<4>(acc, part + int64_t(block) * 4);
    if constexpr (PROD) wave_partials<3>(accp, pk.part + int64_t(block) * 3);
}

template <int ST, int SP, bool G>
__global__ __launch_bounds__(CTHREADS, ST == ST_F64 ? 1 : ((SP & SP_PRODUCT_FLAG) ? 3 : 5)) void k_sweep_c(
    Geometry g, PhysK<typename Store<ST>::T> ph, Slots in, OutSlots out,
    const typename Store<ST>::S *__restrict__ emit, double *__restrict__ part, ProdK<ST> pk) {
    sweep_block_c<ST, SP, G>(g, ph, in, out, emit, part, uint32_t(xcd_block(int(blockIdx.x), int(gridDim.x))), pk);
}

template <int ST, int SP>
__global__ __launch_bounds__(256, ST == ST_F64 ? 1 : (sizeof(typename Store<ST>::S) == 2 ? 5 : 6)) void k_sweep(Geometry g, PhysK<typename Store<ST>::T> ph, Slots in, OutSlots out,
                                                const typename Store<ST>::S *__restrict__ emit,
                                                double *__restrict__ part) {
    sweep_block<ST, SP>(g, ph, in, out, emit, part, uint32_t(xcd_block(int(blockIdx.x), int(gridDim.x))));
}

// Outputs cover the x-rows [row0, row1) (row = z ny + y): voxel v of those
// rows goes to index v - row0 nx, velocity component a to a cs + that index.
template <int ST, bool LOCAL, typename OUT>
__global__ __launch_bounds__(256) void k_fields(Geometry g, PhysK<typename Store<ST>::T> ph,
                                                 Slots in, const typename Store<ST>::S *__restrict__ emit,
                                                 OUT *rho, OUT *vel, OUT *conc, int64_t row0, int64_t row1,
                                                 int64_t cs) {
    using T = typename Store<ST>::T;
    const WaveUnit u = locate(g, uint32_t(xcd_block(int(blockIdx.x), int(gridDim.x))));
    if (!u.valid || u.x >= g.nx || u.row < row0 || u.row >= row1) return;
    T r = 0, ux = 0, uy = 0, uz = 0, c = 0;
    if (u.active) {
        T hC[19], hR[19];
        if (LOCAL) {
#pragma unroll
            for (int i = 0; i < 19; ++i) {
                const typename Store<ST>::P v =
                    static_cast<const typename Store<ST>::P *>(in.p(dslot(i)))[node_elem(g, u.idx)];
                hC[i] = Store<ST>::cv(v.x);
                hR[i] = Store<ST>::cv(v.y);
            }
        } else {
            uint32_t cat_bits;
            pull<ST, -1>(g, ph, in, emit, u, hC, hR, cat_bits);
        }
        const Mom<T> m = moments(ph, hC, hR);
        r = m.rc;
        c = m.rr;
        ux = m.ux;
        uy = m.uy;
        uz = m.uz;
    }
    const int64_t v = (int64_t(u.row) - row0) * g.nx + u.x;
    if (rho) rho[v] = OUT(r);
    if (conc) conc[v] = OUT(c);
    if (vel) {
        vel[v] = OUT(ux);
        vel[cs + v] = OUT(uy);
        vel[2 * cs + v] = OUT(uz);
    }
}

// Initial state: rest equilibrium rho0 / c0 (pre-collision, into `pre`) and
// its collision (into `post`).  Uniform, so every gas node gets the same.
template <int ST>
__global__ __launch_bounds__(256) void k_init(Geometry g, PhysK<typename Store<ST>::T> ph,
                                               typename Store<ST>::S *__restrict__ pre,
                                               typename Store<ST>::S *__restrict__ post) {
    using T = typename Store<ST>::T;
    const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (n >= g.nfp) return;
    using P = typename Store<ST>::P;
    P *pre2 = reinterpret_cast<P *>(pre), *post2 = reinterpret_cast<P *>(post);
    T hC[19], hR[19];
    if (n >= g.nfluid) {
        // padding (the last element of every array holds the normalised
        // reservoir population, which no kernel needs to read)
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            pre2[slot_elem(g, dslot(i)) + node_elem(g, uint32_t(n))] = pop_pair<ST>(T(0), ph.h_inlet);
            post2[slot_elem(g, dslot(i)) + node_elem(g, uint32_t(n))] = pop_pair<ST>(T(0), ph.h_inlet);
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        hC[i] = ph.h0c;
        hR[i] = ph.h0r;
    }
    carrier_shift(ph, hC);
#pragma unroll
    for (int i = 0; i < 19; ++i) pre2[slot_elem(g, dslot(i)) + node_elem(g, uint32_t(n))] = pop_pair<ST>(hC[i], hR[i]);
    const Mom<T> m = moments(ph, hC, hR);
    collide(ph, m, hC, hR);
#pragma unroll
    for (int i = 0; i < 19; ++i) post2[slot_elem(g, dslot(i)) + node_elem(g, uint32_t(n))] = pop_pair<ST>(hC[i], hR[i]);
}

__device__ __forceinline__ uint32_t rank_of(const Geometry &g, int row, int x, bool *fluid) {
    const ChunkInfo &I = g.chunks[int64_t(row) * g.W + (x >> 6)];
    const int b = x & 63;
    *fluid = (I.fluid >> b) & 1u;
    const uint64_t below = b ? (I.fluid & (~0ull >> (64 - b))) : 0ull;
    return I.base + uint32_t(__popcll(below));
}

// Sputtering boundary at each interface node (first line of the sputtering
// equations): In(k) = sum_j f*_j(k - c_j) over its active links was summed by
// the sweep that produced those populations (fixed point, any order); here it
// is read and cleared for the next sweep, added to Acc(k), and re-emitted as
// E(k) = (1 - p_S) In(k) scale(k).  With the product lattice (pi.inacc set)
// In_P(k) is read and cleared the same way, added to Acc_P(k), and the
// product re-emission E_P(k) = (p p_S^R In(k) + (1 - p_S^P) In_P(k)) scale(k)
// is written (second sputtering equation).
struct ProdI {
    void *emit;
    unsigned long long *inacc;
    double *acc;
    double *part;
};

// In(k) from the fixed-point sum of b terms (and clear it).
__device__ __forceinline__ double take_in(unsigned long long *inacc, int64_t k, uint32_t b, double unscale) {
    const unsigned long long raw = glb(inacc)[k] - uint64_t(b) * MAGIC_BITS;
    glb(inacc)[k] = 0ull;
    const long long fixed = static_cast<long long>(raw);
    // a term outside the fixed-point range (|term| >= 2^51 / 2^S) cannot
    // come from a bounded state; report it through the NaN watchdog
    return lbmfx::sum_in_range(fixed) ? double(fixed) * unscale : __builtin_nan("");
}

template <int ST>
__device__ __forceinline__ void interface_block(const PhysK<typename Store<ST>::T> &ph, const Interface &it,
                                                typename Store<ST>::S *__restrict__ emit, double *__restrict__ part,
                                                uint32_t block, const ProdI &pi) {
    using T = typename Store<ST>::T;
    using S = typename Store<ST>::S;
    const int64_t k = int64_t(block) * blockDim.x + threadIdx.x;
    double arrived[1] = {0.0}, arrived_p[1] = {0.0};
    // rounding words of the emission stores: t = exit e (STOCHASTIC), else 0
    // for E(k) and 1 for E_P(k)
    const lbmfx::RoundWords rw = lbmfx::round_words(ph.sr != 0u, ph.sr_key_e, uint32_t(k));
    if (k < it.n && ph.sputter == SP_STOCHASTIC) {
        // one In slot per exit direction; each re-emits (1 - p_S) of its sum
        // along its own exit (stored divided by w_e, like WEIGHTED's E)
        const uint32_t m = glb(it.mask)[k];
        double in = 0.0;
#pragma unroll
        for (int e = 1; e < 19; ++e) {
            if ((m >> opp(e)) & 1u) {
                const uint64_t slot = uint64_t(uint32_t(e - 1)) * uint64_t(it.n) + uint64_t(k);
                const long long fixed = static_cast<long long>(glb(it.inacc)[slot]);
                glb(it.inacc)[slot] = 0ull;
                const double ine = lbmfx::sum_in_range(fixed) ? double(fixed) * ph.in_unscale : __builtin_nan("");
                in += ine;
                st_at(emit, uint32_t(slot) * uint32_t(sizeof(S)),
                      Store<ST>::enc1(T(double(ph.keep) * ine * inv_wgt<double>(e)), rw.at(e)));
            }
        }
        glb(it.acc)[k] += in;
        arrived[0] = in;
    } else if (k < it.n) {
        const uint32_t b = uint32_t(__popc(glb(it.mask)[k]));
        const double in = take_in(it.inacc, k, b, ph.in_unscale);
        glb(it.acc)[k] += in;
        const double scale = glb(it.scale)[k];
        if (ph.sputter != SP_BOUNCEBACK)
            st_at(emit, uint32_t(k) * uint32_t(sizeof(S)), Store<ST>::enc1(T(double(ph.keep) * in * scale), rw.at(0)));
        arrived[0] = in;
        if (pi.inacc) {
            const double inp = take_in(pi.inacc, k, b, ph.in_unscale);
            glb(pi.acc)[k] += inp;
            if (ph.sputter != SP_BOUNCEBACK)
                st_at(static_cast<S *>(pi.emit), uint32_t(k) * uint32_t(sizeof(S)),
                      Store<ST>::enc1(T((double(ph.a_r) * in + double(ph.a_p) * inp) * scale), rw.at(1)));
            arrived_p[0] = inp;
        }
    }
    block_sum<1>(arrived, part + block);
    if (pi.inacc) block_sum<1>(arrived_p, pi.part + block);
}


// Pre-collision populations of both lattices in a box of voxels (the same
// pull as the sweep and the field kernels), as FP64 f_i = w_i (h_i + ref),
// direction-major [19][wz][wy][wx]; solid voxels 0.
template <int ST, bool LOCAL>
__global__ __launch_bounds__(256) void k_populations(Geometry g, PhysK<typename Store<ST>::T> ph, Slots in,
                                                      const typename Store<ST>::S *__restrict__ emit, Window win,
                                                      double *__restrict__ fC, double *__restrict__ fR) {
    using T = typename Store<ST>::T;
    const WaveUnit u = locate(g, uint32_t(xcd_block(int(blockIdx.x), int(gridDim.x))));
    if (!u.valid) return;
    const int wxi = u.x - win.x0, wyi = u.y - win.y0, wzi = u.z - win.z0;
    const bool inside = u.x < g.nx && wxi >= 0 && wxi < win.wx && wyi >= 0 && wyi < win.wy && wzi >= 0 &&
                        wzi < win.wz;
    if (!__builtin_amdgcn_ballot_w64(inside)) return;  // whole wavefront outside the box
    T hC[19], hR[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) hC[i] = hR[i] = T(0);
    if (u.active) {
        if (LOCAL) {
#pragma unroll
            for (int i = 0; i < 19; ++i) {
                const typename Store<ST>::P v =
                    static_cast<const typename Store<ST>::P *>(in.p(dslot(i)))[node_elem(g, u.idx)];
                hC[i] = Store<ST>::cv(v.x);
                hR[i] = Store<ST>::cv(v.y);
            }
        } else {
            uint32_t cat_bits;
            pull<ST, -1>(g, ph, in, emit, u, hC, hR, cat_bits);
        }
        carrier_unshift(ph, hC);  // the populations themselves
    }
    if (!inside) return;
    const int64_t wn = int64_t(win.wx) * win.wy * win.wz;
    const int64_t w = (int64_t(wzi) * win.wy + wyi) * win.wx + wxi;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        fC[i * wn + w] = u.active ? wgt<double>(i) * (double(hC[i]) + double(ph.rref)) : 0.0;
        fR[i * wn + w] = u.active ? wgt<double>(i) * (double(hR[i]) + double(ph.cref)) : 0.0;
    }
}

// In(k) of every interface node from a post-collision population buffer,
// the same fixed-point terms the sweep accumulates (after create and after a
// checkpoint load).
template <int ST>
__global__ __launch_bounds__(256) void k_in_init(Geometry g, PhysK<typename Store<ST>::T> ph, Interface it,
                                                  const typename Store<ST>::S *__restrict__ fin) {
    using T = typename Store<ST>::T;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= it.n) return;
    const uint32_t v = it.vox[k];
    const uint32_t mask = it.mask[k];
    const int x = int(v % uint32_t(g.nx));
    const int row = int(v / uint32_t(g.nx));
    const int y = row % g.ny, z = row / g.ny;
    unsigned long long sum = 0ull, slots[NSLOT];
#pragma unroll
    for (int e = 0; e < NSLOT; ++e) slots[e] = 0ull;
#pragma unroll
    for (int j = 1; j < 19; ++j) {
        if (mask & (1u << j)) {
            int xs = x - CX[j], ys = y - CY[j], zs = z - CZ[j];
            xs = xs < 0 ? xs + g.nx : (xs >= g.nx ? xs - g.nx : xs);
            ys = ys < 0 ? ys + g.ny : (ys >= g.ny ? ys - g.ny : ys);
            zs = zs < 0 ? zs + g.nz : (zs >= g.nz ? zs - g.nz : zs);
            bool fl;
            const uint32_t r = rank_of(g, zs * g.ny + ys, xs, &fl);
            const unsigned long long term =
                in_term<T>(wgt<T>(j), Store<ST>::ld(fin + 2 * (slot_elem(g, dslot(j)) + node_elem(g, r)) + 1), ph.cref,
                           ph.in_scale);
            sum += term;
            if (ph.sputter == SP_STOCHASTIC) {
                const int e = random_exit(ph.step_ctr, ph.seed_lo, ph.seed_hi, v, mask, uint32_t(vcode(j)));
#pragma unroll
                for (int d = 1; d < 19; ++d)
                    if (d == e) slots[d - 1] += term - MAGIC_BITS;
            }
        }
    }
    if (ph.sputter == SP_STOCHASTIC) {
#pragma unroll
        for (int e = 0; e < NSLOT; ++e) it.inacc[uint64_t(uint32_t(e)) * uint64_t(it.n) + uint64_t(k)] = slots[e];
    } else {
        it.inacc[k] = sum;
    }
}

// In_P(k) of every interface node from a product post-collision buffer (one
// unshifted population per element).
template <int ST>
__global__ __launch_bounds__(256) void k_in_init_p(Geometry g, PhysK<typename Store<ST>::T> ph, Interface it,
                                                    const typename Store<ST>::S *__restrict__ finp,
                                                    unsigned long long *__restrict__ inacc) {
    using T = typename Store<ST>::T;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= it.n) return;
    const uint32_t v = it.vox[k];
    const uint32_t mask = it.mask[k];
    const int x = int(v % uint32_t(g.nx));
    const int row = int(v / uint32_t(g.nx));
    const int y = row % g.ny, z = row / g.ny;
    unsigned long long sum = 0ull;
#pragma unroll
    for (int j = 1; j < 19; ++j) {
        if (mask & (1u << j)) {
            int xs = x - CX[j], ys = y - CY[j], zs = z - CZ[j];
            xs = xs < 0 ? xs + g.nx : (xs >= g.nx ? xs - g.nx : xs);
            ys = ys < 0 ? ys + g.ny : (ys >= g.ny ? ys - g.ny : ys);
            zs = zs < 0 ? zs + g.nz : (zs >= g.nz ? zs - g.nz : zs);
            bool fl;
            const uint32_t r = rank_of(g, zs * g.ny + ys, xs, &fl);
            sum += in_term<T>(wgt<T>(j), Store<ST>::ld(finp + slot_elem(g, dslot(j)) + node_elem(g, r)), T(0),
                              ph.in_scale);
        }
    }
    inacc[k] = sum;
}

// Product concentration of every voxel (one thread per voxel): the moments
// of the product populations after streaming finp (LOCAL: of finp itself).
// The pull is written node by node with the same sources as the sweep: y and
// z periodic; x periodic or the reservoir planes (no product at the inlet,
// the copy of plane nx - 1 at the outlet); gas sources; inert sources and a
// solid outlet copy reflect; catalytic sources re-emit E_P(k), or for
// reversal p p_S^R times the reactant plus 1 - p_S^P times the product
// population of the reversed link.  Off the stepping path.
template <int ST, bool LOCAL>
__global__ __launch_bounds__(256) void k_product_field(Geometry g, PhysK<typename Store<ST>::T> ph,
                                                        const typename Store<ST>::S *__restrict__ fin,
                                                        const typename Store<ST>::S *__restrict__ finp,
                                                        const typename Store<ST>::S *__restrict__ emitp,
                                                        double *__restrict__ conc) {
    using T = typename Store<ST>::T;
    const int64_t n = int64_t(g.nx) * g.ny * g.nz;
    const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int x = int(v % g.nx);
    const int row = int(v / g.nx);
    const int y = row % g.ny, z = row / g.ny;
    bool gas;
    const uint32_t me = rank_of(g, row, x, &gas);
    if (!gas) {
        conc[v] = 0.0;
        return;
    }
    const bool xper = ph.species_x == XB_PERIODIC;
    auto popp = [&](int i, uint32_t r) { return Store<ST>::ld(finp + slot_elem(g, dslot(i)) + node_elem(g, r)); };
    auto popr = [&](int i, uint32_t r) {
        return Store<ST>::ld(fin + 2 * (slot_elem(g, dslot(i)) + node_elem(g, r)) + 1);
    };
    double rho = 0.0;
#pragma unroll 1
    for (int i = 0; i < 19; ++i) {
        T h;
        if (LOCAL || i == 0) {
            h = popp(i, me);
        } else {
            int xs = x - CX[i], ys = y - CY[i], zs = z - CZ[i];
            ys = ys < 0 ? ys + g.ny : (ys >= g.ny ? ys - g.ny : ys);
            zs = zs < 0 ? zs + g.nz : (zs >= g.nz ? zs - g.nz : zs);
            if (xper) xs = xs < 0 ? xs + g.nx : (xs >= g.nx ? xs - g.nx : xs);
            const int srow = zs * g.ny + ys;
            if (xs < 0) {
                h = T(0);  // inlet ghost: no product injected
            } else if (xs >= g.nx) {
                bool fl;
                const uint32_t r = rank_of(g, srow, g.nx - 1, &fl);
                h = fl ? popp(i, r) : popp(opp(i), me);
            } else {
                const ChunkInfo &I = g.chunks[int64_t(srow) * g.W + (xs >> 6)];
                const int b = xs & 63;
                const uint64_t below = b ? (~0ull >> (64 - b)) : 0ull;
                if ((I.fluid >> b) & 1u) {
                    h = popp(i, I.base + uint32_t(__popcll(I.fluid & below)));
                } else if (!((I.cat >> b) & 1u)) {
                    h = popp(opp(i), me);
                } else if (ph.sputter == SP_BOUNCEBACK) {
                    h = ph.a_r * (popr(opp(i), me) + ph.cref) + ph.a_p * popp(opp(i), me);
                } else {
                    const uint32_t k = I.ibase + uint32_t(__popcll(I.cat & below));
                    const T e = Store<ST>::ld(emitp + k);
                    h = ph.sputter == SP_UNIFORM ? e * inv_wgt<T>(i) : e;
                }
            }
        }
        rho += double(wgt<T>(i) * h);
    }
    conc[v] = rho;
}

// phi[x] = sum over the (y, z) plane of conc * u_x: block x, rows strided
// over the threads, then a fixed tree.
__global__ __launch_bounds__(256) void k_flux_profile(int nx, int64_t rows, const double *__restrict__ conc,
                                                       const double *__restrict__ ux, double *__restrict__ phi) {
    __shared__ double sh[256];
    const int x = int(blockIdx.x);
    double s = 0.0;
    for (int64_t r = threadIdx.x; r < rows; r += blockDim.x) s += conc[r * nx + x] * ux[r * nx + x];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (int(threadIdx.x) < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) phi[x] = sh[0];
}

// Fixed-order sum over rows [r0, r1) of column `col` of a row-major
// [n][ncol] partial array, by the whole block (thread-strided, then a tree).
__device__ double column_sum(const double *p, int64_t r0, int64_t r1, int ncol, int col) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) s += p[r * ncol + col];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (int(threadIdx.x) < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double out = sh[0];
    __syncthreads();
    return out;
}

// First stage of the totals: block b folds its contiguous slice of rows of
// each partial array into one row of `out` (fixed order, so deterministic).
// psp / pip: the product partials (3 per sweep block, 1 per interface
// block), or null without the product lattice (its slots stay 0).
__device__ void fold_block(const double *ps, int64_t ns, const double *pi, int64_t ni, double *out, int64_t b,
                           int64_t nb, const double *psp = nullptr, const double *pip = nullptr) {
    auto slice = [&](int64_t n, int64_t *r0, int64_t *r1) {
        const int64_t per = (n + nb - 1) / nb;
        *r0 = b * per < n ? b * per : n;
        *r1 = (b + 1) * per < n ? (b + 1) * per : n;
    };
    int64_t r0, r1;
    double v[NPART];
    slice(ns, &r0, &r1);
    v[PART_MASS_C] = column_sum(ps, r0, r1, 4, 0);
    v[PART_MASS_R] = column_sum(ps, r0, r1, 4, 1);
    v[PART_INFLUX] = column_sum(ps, r0, r1, 4, 2);
    v[PART_OUTFLUX] = column_sum(ps, r0, r1, 4, 3);
    if (psp) {
        v[PART_MASS_P] = column_sum(psp, r0, r1, 3, 0);
        v[PART_POUT_IN] = column_sum(psp, r0, r1, 3, 1);
        v[PART_POUT_OUT] = column_sum(psp, r0, r1, 3, 2);
    } else {
        v[PART_MASS_P] = v[PART_POUT_IN] = v[PART_POUT_OUT] = 0.0;
    }
    slice(ni, &r0, &r1);
    v[PART_IN] = column_sum(pi, r0, r1, 1, 0);
    v[PART_IN_P] = pip ? column_sum(pip, r0, r1, 1, 0) : 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NPART; ++k) out[b * NPART + k] = v[k];
}


// `product`: also sum the product slots into the product totals (p_stick_p =
// p_S^P); without it only the first NPART_BASE slots are read.
__device__ void reduce_block(const double *folded, int64_t nb, double p, double p_stick, DevTotals *tot,
                             bool product = false, double p_stick_p = 0.0) {
    double v[NPART];
    const int nk = product ? NPART : NPART_BASE;
    for (int k = 0; k < NPART; ++k) v[k] = k < nk ? column_sum(folded, 0, nb, NPART, k) : 0.0;
    if (threadIdx.x == 0) {
        if (product) {
            tot->mass_product = v[PART_MASS_P];
            tot->lost_product += p_stick_p * v[PART_IN_P];
            tot->product_out_inlet += v[PART_POUT_IN];
            tot->product_out_outlet += v[PART_POUT_OUT];
        }
        tot->mass_gas = v[PART_MASS_C];
        tot->mass_species = v[PART_MASS_R];
        tot->converted += p * p_stick * v[PART_IN];
        tot->lost += (1.0 - p) * p_stick * v[PART_IN];
        tot->influx += v[PART_INFLUX];
        tot->outflux += v[PART_OUTFLUX];
        tot->step += 1;
        double all = 0.0;
        for (int k = 0; k < nk; ++k) all += v[k];
        if (!(all - all == 0.0)) tot->nonfinite = 1;
    }
}


// Everything of a step but the sweep, in one launch: the interface of step t
// (the first `iface_blocks` blocks), the first reduction stage of step t - 1
// (the next `fold_blocks`, 0 or FOLD_BLOCKS) and the final stage of step
// t - 2 (one last block, when `reduce`).  The parts touch disjoint buffers
// (interface partials and fold outputs alternate with the step's parity), and
// each runs exactly the code of its own kernel, so the totals are the same.
// The product lattice's parts of a front launch (all null without it).
struct ProdFront {
    ProdI iface;             // interface of step t (iface.part: its partials)
    const double *ps;        // sweep P partials of step t - 1
    const double *pi_prev;   // interface P partials of step t - 1
    double p_stick;          // p_S^P
    int32_t on, pad;
};

template <int ST>
__global__ __launch_bounds__(256) void k_front(PhysK<typename Store<ST>::T> ph, Interface it,
                                                typename Store<ST>::S *__restrict__ emit, double *pi_now,
                                                const double *ps, int64_t ns, const double *pi_prev, int64_t ni,
                                                double *fold_prev, const double *fold_prev2, double p, double p_stick,
                                                DevTotals *tot, int32_t iface_blocks, int32_t fold_blocks,
                                                ProdFront pf) {
    const int32_t b = int32_t(blockIdx.x);
    if (b < iface_blocks) {
        interface_block<ST>(ph, it, emit, pi_now, uint32_t(b), pf.iface);
    } else if (b - iface_blocks < fold_blocks) {
        fold_block(ps, ns, pi_prev, ni, fold_prev, b - iface_blocks, FOLD_BLOCKS, pf.on ? pf.ps : nullptr,
                   pf.on ? pf.pi_prev : nullptr);
    } else {
        reduce_block(fold_prev2, FOLD_BLOCKS, p, p_stick, tot, pf.on != 0, pf.p_stick);
    }
}

// ---------------------------------------------------------------------------
// Batched kernels: one launch covers every sample of a batch.  Each sample
// owns a contiguous range of logical blocks (first block in its record); a
// per-block table names the sample, and the block reads that sample's
// geometry, physics and buffers from its record with scalar loads.  A
// sample's blocks run exactly the code and partial layout of its
// single-sample launch, so its results are bit-identical to those.

template <int ST>
struct SampleK {
    Geometry g;
    Interface it;
    PhysK<typename Store<ST>::T> ph;
    Slots pop[2];  // population buffers A and B
    typename Store<ST>::S *emit;
    double *part_sweep, *part_iface;
    uint32_t block0, iblock0;  // first logical sweep / interface block of the sample
};

template <int ST, int SP>
__global__ __launch_bounds__(256) void k_sweep_batch(const SampleK<ST> *__restrict__ smp,
                                                      const uint32_t *__restrict__ block_sample, int parity) {
    const uint32_t b = uint32_t(xcd_block(int(blockIdx.x), int(gridDim.x)));
    const SampleK<ST> &d = smp[__builtin_amdgcn_readfirstlane(block_sample[b])];
    const Slots &in = d.pop[parity];
    const OutSlots &out = reinterpret_cast<const OutSlots &>(d.pop[1 - parity]);
    sweep_block<ST, SP>(d.g, d.ph, in, out, d.emit, d.part_sweep, b - d.block0);
}

template <int ST, int SP, bool G>
__global__ __launch_bounds__(CTHREADS, ST == ST_F64 ? 1 : 5) void k_sweep_batch_c(const SampleK<ST> *__restrict__ smp,
                                                        const uint32_t *__restrict__ block_sample, int parity) {
    const uint32_t b = uint32_t(xcd_block(int(blockIdx.x), int(gridDim.x)));
    const SampleK<ST> &d = smp[__builtin_amdgcn_readfirstlane(block_sample[b])];
    const Slots &in = d.pop[parity];
    const OutSlots &out = reinterpret_cast<const OutSlots &>(d.pop[1 - parity]);
    sweep_block_c<ST, SP, G>(d.g, d.ph, in, out, d.emit, d.part_sweep, b - d.block0, ProdK<ST>{});
}

template <int ST>
__global__ __launch_bounds__(256) void k_interface_batch(const SampleK<ST> *__restrict__ smp,
                                                          const uint32_t *__restrict__ block_sample) {
    const uint32_t b = blockIdx.x;
    const SampleK<ST> &d = smp[__builtin_amdgcn_readfirstlane(block_sample[b])];
    interface_block<ST>(d.ph, d.it, d.emit, d.part_iface, b - d.iblock0, ProdI{});
}

__global__ __launch_bounds__(256) void k_fold_batch(const ReduceK *__restrict__ r) {
    const ReduceK &d = r[blockIdx.y];
    fold_block(d.ps, d.ns, d.pi, d.ni, d.fold, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void k_reduce_batch(const ReduceK *__restrict__ r) {
    const ReduceK &d = r[blockIdx.x];
    reduce_block(d.fold, FOLD_BLOCKS, d.p, d.p_stick, d.tot);
}

// The sweep template code of a sputter mode and species x-boundary.
int sweep_code(int sputter, int species_x) { return sputter | (species_x == XB_INFLOW ? SP_INFLOW_FLAG : 0); }

template <typename F>
hipError_t dispatch_sp(int code, F &&f) {
    switch (code) {
        case SP_UNIFORM: return f(std::integral_constant<int, SP_UNIFORM>{});
        case SP_WEIGHTED: return f(std::integral_constant<int, SP_WEIGHTED>{});
        case SP_BOUNCEBACK: return f(std::integral_constant<int, SP_BOUNCEBACK>{});
        case SP_UNIFORM | SP_INFLOW_FLAG: return f(std::integral_constant<int, SP_UNIFORM | SP_INFLOW_FLAG>{});
        case SP_WEIGHTED | SP_INFLOW_FLAG: return f(std::integral_constant<int, SP_WEIGHTED | SP_INFLOW_FLAG>{});
        case SP_BOUNCEBACK | SP_INFLOW_FLAG: return f(std::integral_constant<int, SP_BOUNCEBACK | SP_INFLOW_FLAG>{});
        case SP_STOCHASTIC: return f(std::integral_constant<int, SP_STOCHASTIC>{});
        case SP_STOCHASTIC | SP_INFLOW_FLAG: return f(std::integral_constant<int, SP_STOCHASTIC | SP_INFLOW_FLAG>{});
        default: return hipErrorInvalidValue;
    }
}

// The diffuse-wall codes (single-context sweeps).
template <typename F>
hipError_t dispatch_sp_diffuse(int code, F &&f) {
    constexpr int D = SP_DIFFUSE_FLAG, I = SP_INFLOW_FLAG;
    switch (code) {
        case SP_UNIFORM: return f(std::integral_constant<int, D | SP_UNIFORM>{});
        case SP_WEIGHTED: return f(std::integral_constant<int, D | SP_WEIGHTED>{});
        case SP_BOUNCEBACK: return f(std::integral_constant<int, D | SP_BOUNCEBACK>{});
        case SP_STOCHASTIC: return f(std::integral_constant<int, D | SP_STOCHASTIC>{});
        case SP_UNIFORM | I: return f(std::integral_constant<int, D | I | SP_UNIFORM>{});
        case SP_WEIGHTED | I: return f(std::integral_constant<int, D | I | SP_WEIGHTED>{});
        case SP_BOUNCEBACK | I: return f(std::integral_constant<int, D | I | SP_BOUNCEBACK>{});
        case SP_STOCHASTIC | I: return f(std::integral_constant<int, D | I | SP_STOCHASTIC>{});
        default: return hipErrorInvalidValue;
    }
}

// The product-lattice codes (node-compact sweep only).
template <typename F>
hipError_t dispatch_sp_product(int code, F &&f) {
    constexpr int P = SP_PRODUCT_FLAG, I = SP_INFLOW_FLAG;
    switch (code) {
        case SP_UNIFORM: return f(std::integral_constant<int, P | SP_UNIFORM>{});
        case SP_WEIGHTED: return f(std::integral_constant<int, P | SP_WEIGHTED>{});
        case SP_BOUNCEBACK: return f(std::integral_constant<int, P | SP_BOUNCEBACK>{});
        case SP_UNIFORM | I: return f(std::integral_constant<int, P | I | SP_UNIFORM>{});
        case SP_WEIGHTED | I: return f(std::integral_constant<int, P | I | SP_WEIGHTED>{});
        case SP_BOUNCEBACK | I: return f(std::integral_constant<int, P | I | SP_BOUNCEBACK>{});
        default: return hipErrorInvalidValue;
    }
}

template <typename F>
hipError_t dispatch(int storage, F &&f) {
    switch (storage) {
        case ST_F32: return f(std::integral_constant<int, ST_F32>{});
        case ST_F16: return f(std::integral_constant<int, ST_F16>{});
        case ST_BF16: return f(std::integral_constant<int, ST_BF16>{});
        case ST_F64: return f(std::integral_constant<int, ST_F64>{});
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int storage_bytes(int storage) {
    switch (storage) {
        case ST_F32: return 4;
        case ST_F16: return 2;
        case ST_BF16: return 2;
        case ST_F64: return 8;
        default: return 0;
    }
}

// Sweep grids are padded to a multiple of 8 blocks (the padding blocks find
// no work and add zero partials) so that xcd_block can give every XCD one
// contiguous range of the traversal.
int64_t sweep_blocks(const Geometry &g) { return ((int64_t(g.units) + 3) / 4 + 7) / 8 * 8; }

void build_order(int nx, int ny, int nz, int ytile, uint32_t *order) {
    const int W = (nx + 63) / 64;
    size_t k = 0;
    for (int y0 = 0; y0 < ny; y0 += ytile)
        for (int z = 0; z < nz; ++z)
            for (int y = y0; y < y0 + ytile && y < ny; ++y)
                for (int c = 0; c < W; ++c) order[k++] = uint32_t(y) | (uint32_t(z) << 12) | (uint32_t(c) << 24);
}
int64_t interface_blocks(int64_t n) { return n > 0 ? (n + 255) / 256 : 0; }

hipError_t launch_init(const Geometry &g, const Physics &ph, void *pre, void *post, hipStream_t s) {
    return dispatch(ph.storage, [&](auto st) {
        constexpr int ST = decltype(st)::value;
        using SS = typename Store<ST>::S;
        using T = typename Store<ST>::T;
        const int64_t blocks = (g.nfp + 255) / 256;
        hipLaunchKernelGGL(k_init<ST>, dim3(unsigned(blocks)), dim3(256), 0, s, g, to_kernel<T>(ph),
                           static_cast<SS *>(pre), static_cast<SS *>(post));
        return hipGetLastError();
    });
}

hipError_t launch_in_init(const Geometry &g, const Physics &ph, const Interface &it, const void *fin, hipStream_t s) {
    const int64_t blocks = interface_blocks(it.n);
    if (blocks == 0) return hipSuccess;
    return dispatch(ph.storage, [&](auto st) {
        constexpr int ST = decltype(st)::value;
        using SS = typename Store<ST>::S;
        using T = typename Store<ST>::T;
        hipLaunchKernelGGL(k_in_init<ST>, dim3(unsigned(blocks)), dim3(256), 0, s, g, to_kernel<T>(ph), it,
                           static_cast<const SS *>(fin));
        return hipGetLastError();
    });
}

template <int ST>
Slots slots_of(const Geometry &g, const void *buf) {
    Slots sl;
    using S = typename Store<ST>::S;
    sl.base = static_cast<const char *>(buf);
    sl.stride = uint32_t(uint64_t(g.lay_ss) * 2 * sizeof(S));
    sl.pad = 0;
    return sl;
}

hipError_t launch_sweep(const Geometry &g, const Physics &ph, const void *fin, void *fout, const void *emit,
                        double *part, hipStream_t s) {
    return dispatch(ph.storage, [&](auto st) {
        constexpr int ST = decltype(st)::value;
        using SS = typename Store<ST>::S;
        using T = typename Store<ST>::T;
        const Slots in = slots_of<ST>(g, fin);
        OutSlots out;
        out.base = static_cast<char *>(fout);
        out.stride = uint32_t(uint64_t(g.lay_ss) * 2 * sizeof(SS));
        out.pad = 0;
        const dim3 grid(unsigned(sweep_blocks(g))), block(256);
        const SS *e = static_cast<const SS *>(emit);
        const PhysK<T> k = to_kernel<T>(ph);
        auto go = [&](auto sp) {
            hipLaunchKernelGGL((k_sweep<ST, decltype(sp)::value>), grid, block, 0, s, g, k, in, out, e, part);
            return hipGetLastError();
        };
        if (ph.wall_diffuse != 0.0) return dispatch_sp_diffuse(sweep_code(ph.sputter, ph.species_x), go);
        return dispatch_sp(sweep_code(ph.sputter, ph.species_x), go);
    });
}

int64_t sweep_blocks_c(const Geometry &g) { return (int64_t(g.nwaves) + 7) / 8 * 8; }

bool emission_gather_applies(int storage, int sputter, bool product) {
    return (storage == ST_F32 || storage == ST_F64) && !product && (sputter == SP_UNIFORM || sputter == SP_WEIGHTED);
}

hipError_t launch_sweep_c(const Geometry &g, const Physics &ph, const void *fin, void *fout, const void *emit,
                          double *part, hipStream_t s, const ProdStep *prod) {
    return dispatch(ph.storage, [&](auto st) {
        constexpr int ST = decltype(st)::value;
        using SS = typename Store<ST>::S;
        using T = typename Store<ST>::T;
        const Slots in = slots_of<ST>(g, fin);
        OutSlots out;
        out.base = static_cast<char *>(fout);
        out.stride = uint32_t(uint64_t(g.lay_ss) * 2 * sizeof(SS));
        out.pad = 0;
        const dim3 grid(static_cast<unsigned>(sweep_blocks_c(g))), block(CTHREADS);
        const SS *e = static_cast<const SS *>(emit);
        const PhysK<T> k = to_kernel<T>(ph);
        if (prod) {
            ProdK<ST> pk{};
            pk.in.base = static_cast<const char *>(prod->fin);
            pk.in.stride = uint32_t(uint64_t(g.lay_ss) * sizeof(SS));
            pk.out.base = static_cast<char *>(prod->fout);
            pk.out.stride = pk.in.stride;
            pk.emit = static_cast<const SS *>(prod->emit);
            pk.inacc = prod->inacc;
            pk.part = prod->part_sweep;
            return dispatch_sp_product(sweep_code(ph.sputter, ph.species_x), [&](auto sp) {
                hipLaunchKernelGGL((k_sweep_c<ST, decltype(sp)::value, false>), grid, block, 0, s, g, k, in, out, e,
                                   part, pk);
                return hipGetLastError();
            });
        }
        const bool gather = ph.emission_gather != 0;
        auto go = [&](auto sp) {
            constexpr int SP = decltype(sp)::value;
            if constexpr (gather_applies<ST, SP>()) {
                if (gather) {
                    hipLaunchKernelGGL((k_sweep_c<ST, SP, true>), grid, block, 0, s, g, k, in, out, e, part,
                                       ProdK<ST>{});
                    return hipGetLastError();
                }
            }
            hipLaunchKernelGGL((k_sweep_c<ST, SP, false>), grid, block, 0, s, g, k, in, out, e, part, ProdK<ST>{});
            return hipGetLastError();
        };
        if (ph.wall_diffuse != 0.0) return dispatch_sp_diffuse(sweep_code(ph.sputter, ph.species_x), go);
        return dispatch_sp(sweep_code(ph.sputter, ph.species_x), go);
    });
}

hipError_t launch_fields(const Geometry &g, const Physics &ph, const void *fin, const void *emit, int mode, void *rho,
                         void *u, void *conc, bool out_f64, hipStream_t s) {
    const int64_t rows = int64_t(g.ny) * g.nz;
    return launch_fields_rows(g, ph, fin, emit, mode, rho, u, conc, out_f64, 0, rows, rows * g.nx, s);
}

hipError_t launch_fields_rows(const Geometry &g, const Physics &ph, const void *fin, const void *emit, int mode,
                              void *rho, void *u, void *conc, bool out_f64, int64_t row0, int64_t row1, int64_t cs,
                              hipStream_t s) {
    return dispatch(ph.storage, [&](auto st) {
        constexpr int ST = decltype(st)::value;
        using SS = typename Store<ST>::S;
        using T = typename Store<ST>::T;
        const dim3 grid(unsigned(sweep_blocks(g))), block(256);
        const Slots f = slots_of<ST>(g, fin);
        const SS *e = static_cast<const SS *>(emit);
        const PhysK<T> k = to_kernel<T>(ph);
        if (out_f64) {
            double *a = static_cast<double *>(rho), *b = static_cast<double *>(u), *c = static_cast<double *>(conc);
            if (mode == 2)
                hipLaunchKernelGGL((k_fields<ST, true, double>), grid, block, 0, s, g, k, f, e, a, b, c, row0, row1,
                                   cs);
            else
                hipLaunchKernelGGL((k_fields<ST, false, double>), grid, block, 0, s, g, k, f, e, a, b, c, row0, row1,
                                   cs);
        } else {
            float *a = static_cast<float *>(rho), *b = static_cast<float *>(u), *c = static_cast<float *>(conc);
            if (mode == 2)
                hipLaunchKernelGGL((k_fields<ST, true, float>), grid, block, 0, s, g, k, f, e, a, b, c, row0, row1,
                                   cs);
            else
                hipLaunchKernelGGL((k_fields<ST, false, float>), grid, block, 0, s, g, k, f, e, a, b, c, row0, row1,
                                   cs);
        }
        return hipGetLastError();
    });
}

hipError_t launch_populations(const Geometry &g, const Physics &ph, const void *fin, const void *emit, int mode,
                              const Window &win, double *fC, double *fR, hipStream_t s) {
    return dispatch(ph.storage, [&](auto st) {
        constexpr int ST = decltype(st)::value;
        using SS = typename Store<ST>::S;
        using T = typename Store<ST>::T;
        const dim3 grid(unsigned(sweep_blocks(g))), block(256);
        const Slots f = slots_of<ST>(g, fin);
        const SS *e = static_cast<const SS *>(emit);
        const PhysK<T> k = to_kernel<T>(ph);
        if (mode == 2)
            hipLaunchKernelGGL((k_populations<ST, true>), grid, block, 0, s, g, k, f, e, win, fC, fR);
        else
            hipLaunchKernelGGL((k_populations<ST, false>), grid, block, 0, s, g, k, f, e, win, fC, fR);
        return hipGetLastError();
    });
}

hipError_t launch_front(const Physics &ph, const Interface &it, void *emit, int64_t iface_blocks, double *pi_now,
                        const double *ps, int64_t ns, const double *pi_prev, int64_t ni, double *fold_prev,
                        bool fold, const double *fold_prev2, bool reduce, DevTotals *tot, hipStream_t s,
                        const ProdStep *prod) {
    const int64_t blocks = iface_blocks + (fold ? FOLD_BLOCKS : 0) + (reduce ? 1 : 0);
    if (blocks == 0) return hipSuccess;
    ProdFront pf{};
    if (prod) {
        pf.on = 1;
        pf.p_stick = ph.p_stick_product;
        pf.iface.emit = prod->emit;
        pf.iface.inacc = iface_blocks > 0 ? prod->inacc : nullptr;
        pf.iface.acc = prod->acc;
        pf.iface.part = prod->pi_now;
        pf.ps = prod->part_sweep;
        pf.pi_prev = prod->pi_prev;
    }
    return dispatch(ph.storage, [&](auto st) {
        constexpr int ST = decltype(st)::value;
        using SS = typename Store<ST>::S;
        using T = typename Store<ST>::T;
        hipLaunchKernelGGL(k_front<ST>, dim3(unsigned(blocks)), dim3(256), 0, s, to_kernel<T>(ph), it,
                           static_cast<SS *>(emit), pi_now, ps, ns, pi_prev, ni, fold_prev, fold_prev2, ph.p,
                           ph.p_stick, tot, int32_t(iface_blocks), int32_t(fold ? FOLD_BLOCKS : 0), pf);
        return hipGetLastError();
    });
}

hipError_t launch_in_init_product(const Geometry &g, const Physics &ph, const Interface &it, const void *finP,
                                  unsigned long long *inacc, hipStream_t s) {
    const int64_t blocks = interface_blocks(it.n);
    if (blocks == 0) return hipSuccess;
    return dispatch(ph.storage, [&](auto st) {
        constexpr int ST = decltype(st)::value;
        using SS = typename Store<ST>::S;
        using T = typename Store<ST>::T;
        hipLaunchKernelGGL(k_in_init_p<ST>, dim3(unsigned(blocks)), dim3(256), 0, s, g, to_kernel<T>(ph), it,
                           static_cast<const SS *>(finP), inacc);
        return hipGetLastError();
    });
}

hipError_t launch_product_field(const Geometry &g, const Physics &ph, const void *fin, const void *finP,
                                const void *emitP, int mode, double *concP, hipStream_t s) {
    const int64_t n = int64_t(g.nx) * g.ny * g.nz;
    const dim3 grid(unsigned((n + 255) / 256)), block(256);
    return dispatch(ph.storage, [&](auto st) {
        constexpr int ST = decltype(st)::value;
        using SS = typename Store<ST>::S;
        using T = typename Store<ST>::T;
        const SS *a = static_cast<const SS *>(fin), *b = static_cast<const SS *>(finP),
                 *e = static_cast<const SS *>(emitP);
        if (mode == 2)
            hipLaunchKernelGGL((k_product_field<ST, true>), grid, block, 0, s, g, to_kernel<T>(ph), a, b, e, concP);
        else
            hipLaunchKernelGGL((k_product_field<ST, false>), grid, block, 0, s, g, to_kernel<T>(ph), a, b, e, concP);
        return hipGetLastError();
    });
}

hipError_t launch_flux_profile(const Geometry &g, const double *concP, const double *u, double *phi, hipStream_t s) {
    hipLaunchKernelGGL(k_flux_profile, dim3(unsigned(g.nx)), dim3(256), 0, s, g.nx, int64_t(g.ny) * g.nz, concP, u,
                       phi);
    return hipGetLastError();
}

size_t batch_record_bytes(int storage) {
    switch (storage) {
        case ST_F32: return sizeof(SampleK<ST_F32>);
        case ST_F16: return sizeof(SampleK<ST_F16>);
        case ST_BF16: return sizeof(SampleK<ST_BF16>);
        case ST_F64: return sizeof(SampleK<ST_F64>);
        default: return 0;
    }
}

hipError_t batch_upload(int storage, const BatchSample *smp, int n, void *d_records, hipStream_t s) {
    return dispatch(storage, [&](auto st) {
        constexpr int ST = decltype(st)::value;
        using SS = typename Store<ST>::S;
        using T = typename Store<ST>::T;
        std::vector<SampleK<ST>> rec(static_cast<size_t>(n));
        for (int i = 0; i < n; ++i) {
            SampleK<ST> &r = rec[size_t(i)];
            std::memset(static_cast<void *>(&r), 0, sizeof(r));
            r.g = smp[i].g;
            r.it = smp[i].it;
            r.ph = to_kernel<T>(smp[i].ph);
            r.pop[0] = slots_of<ST>(smp[i].g, smp[i].pop[0]);
            r.pop[1] = slots_of<ST>(smp[i].g, smp[i].pop[1]);
            r.emit = static_cast<SS *>(smp[i].emit);
            r.part_sweep = smp[i].part_sweep;
            r.part_iface = smp[i].part_iface;
            r.block0 = smp[i].block0;
            r.iblock0 = smp[i].iblock0;
        }
        hipError_t e = hipMemcpyAsync(d_records, rec.data(), rec.size() * sizeof(SampleK<ST>), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        return e;
    });
}

hipError_t launch_batch_sweep(int storage, int sputter, int species_x, bool compact, bool gather,
                              const void *d_records, const uint32_t *sweep_sample, int64_t sweep_blocks_total,
                              int parity, hipStream_t s) {
    return dispatch(storage, [&](auto st) {
        constexpr int ST = decltype(st)::value;
        const SampleK<ST> *rec = static_cast<const SampleK<ST> *>(d_records);
        const dim3 grid(static_cast<unsigned>(sweep_blocks_total)), block(compact ? CTHREADS : 256u);
        return dispatch_sp(sweep_code(sputter, species_x), [&](auto sp) {
            constexpr int SP = decltype(sp)::value;
            if constexpr (gather_applies<ST, SP>()) {
                if (compact && gather) {
                    hipLaunchKernelGGL((k_sweep_batch_c<ST, SP, true>), grid, block, 0, s, rec, sweep_sample, parity);
                    return hipGetLastError();
                }
            }
            if (compact)
                hipLaunchKernelGGL((k_sweep_batch_c<ST, SP, false>), grid, block, 0, s, rec, sweep_sample, parity);
            else
                hipLaunchKernelGGL((k_sweep_batch<ST, SP>), grid, block, 0, s, rec, sweep_sample, parity);
            return hipGetLastError();
        });
    });
}

hipError_t launch_batch_step(int storage, int sputter, int species_x, bool compact, bool gather, const void *d_records,
                             const uint32_t *sweep_sample, int64_t sweep_blocks_total, const uint32_t *iface_sample,
                             int64_t iface_blocks_total, const ReduceK *d_reduce, int n, int parity, hipStream_t s,
                             hipEvent_t sweep_start, hipEvent_t sweep_stop) {
    return dispatch(storage, [&](auto st) {
        constexpr int ST = decltype(st)::value;
        const SampleK<ST> *rec = static_cast<const SampleK<ST> *>(d_records);
        if (iface_blocks_total > 0) {
            hipLaunchKernelGGL(k_interface_batch<ST>, dim3(unsigned(iface_blocks_total)), dim3(256), 0, s, rec,
                               iface_sample);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        hipError_t e = sweep_start ? hipEventRecord(sweep_start, s) : hipSuccess;
        if (e != hipSuccess) return e;
        e = launch_batch_sweep(storage, sputter, species_x, compact, gather, d_records, sweep_sample,
                               sweep_blocks_total, parity, s);
        if (e != hipSuccess) return e;
        e = sweep_stop ? hipEventRecord(sweep_stop, s) : hipSuccess;
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_fold_batch, dim3(FOLD_BLOCKS, unsigned(n)), dim3(256), 0, s, d_reduce);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_reduce_batch, dim3(unsigned(n)), dim3(256), 0, s, d_reduce);
        return hipGetLastError();
    });
}

// ------------------------------------------------ allocation-free entry --
// Scratch of lbm_fields_noalloc: a bounce buffer for field rows, in every
// GPU's copy of the code object, held until the process ends.  Host code
// never uses the array's name as an address (in host code it is a stand-in
// for the device object): scratch_address asks the runtime for the address of
// the current device's copy, once per device, and callers pass that pointer.
static __device__ __align__(256) double scratch[FIELDS_SCRATCH_DOUBLES];

hipError_t scratch_address(int device, double **out) {
    static std::mutex mu;
    static double *addr[MAX_SCRATCH_DEVICES] = {};
    if (device < 0 || device >= MAX_SCRATCH_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // the lookup needs that device current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = static_cast<double *>(p);
    }
    *out = addr[device];
    return hipSuccess;
}

// ------------------------------------------------- HBM copy reference --
// The streaming copy the sweep's bandwidth is compared with: one 16-byte
// element per thread, non-temporal load and store (on MI355X the fastest of
// the copy forms tried: more elements per thread, or cached accesses, run
// slower).  Not part of the method.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_stream_copy(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                                                      uint64_t n) {
    const uint64_t i = uint64_t(blockIdx.x) * 256u + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

hipError_t launch_stream_copy(void *dst, const void *src, size_t bytes, hipStream_t s) {
    const uint64_t n = bytes / 16u;
    if (n == 0) return hipSuccess;
    const uint64_t blocks = (n + 255u) / 256u;
    if (blocks > 0xffffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_stream_copy, dim3(unsigned(blocks)), dim3(256), 0, s, static_cast<const u32x4 *>(src),
                       static_cast<u32x4 *>(dst), n);
    return hipGetLastError();
}

// ---------------------------------------- pull-streaming reference --
// The data movement of the sweep without its arithmetic: one pull-streaming
// pass of D3Q19 over a dense periodic nx x ny x nz lattice stored in the
// sweep's blocked layout (the 19 slots of 64 consecutive nodes contiguous).
// Node n = x + nx (y + ny z) reads element i of its upwind neighbour
// (x - c_ix, y - c_iy, z - c_iz) and writes it to its own slot i, one
// non-temporal load and store per direction and node.  A population pair of
// the sweep is one element E (4, 8 or 16 bytes).  Not part of the method.
template <typename E>
__global__ __launch_bounds__(256) void k_stream_pull(const E *__restrict__ src, E *__restrict__ dst, int nx, int ny,
                                                     int nz) {
    const int x = int(blockIdx.x) * 256 + int(threadIdx.x), y = int(blockIdx.y), z = int(blockIdx.z);
    if (x >= nx) return;
    const uint32_t n = uint32_t(x) + uint32_t(nx) * (uint32_t(y) + uint32_t(ny) * uint32_t(z));
    const uint32_t own = (n >> 6) * (19u * 64u) + (n & 63u);
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        int xs = x - CX[i], ys = y - CY[i], zs = z - CZ[i];
        xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
        ys = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
        zs = zs < 0 ? zs + nz : (zs >= nz ? zs - nz : zs);
        const uint32_t m = uint32_t(xs) + uint32_t(nx) * (uint32_t(ys) + uint32_t(ny) * uint32_t(zs));
        const E v = __builtin_nontemporal_load(src + (m >> 6) * (19u * 64u) + uint32_t(i) * 64u + (m & 63u));
        __builtin_nontemporal_store(v, dst + own + uint32_t(i) * 64u);
    }
}

uint64_t stream_pull_elements(int nx, int ny, int nz) {
    const uint64_t n = uint64_t(nx) * uint64_t(ny) * uint64_t(nz);
    return (n + 63u) / 64u * 64u * 19u;
}

hipError_t launch_stream_pull(void *dst, const void *src, int nx, int ny, int nz, int pair_bytes, hipStream_t s) {
    const dim3 grid(unsigned((nx + 255) / 256), unsigned(ny), unsigned(nz)), block(256);
    switch (pair_bytes) {
    case 4:
        hipLaunchKernelGGL(k_stream_pull<uint32_t>, grid, block, 0, s, static_cast<const uint32_t *>(src),
                           static_cast<uint32_t *>(dst), nx, ny, nz);
        break;
    case 8:
        hipLaunchKernelGGL(k_stream_pull<uint64_t>, grid, block, 0, s, static_cast<const uint64_t *>(src),
                           static_cast<uint64_t *>(dst), nx, ny, nz);
        break;
    case 16:
        hipLaunchKernelGGL(k_stream_pull<u32x4>, grid, block, 0, s, static_cast<const u32x4 *>(src),
                           static_cast<u32x4 *>(dst), nx, ny, nz);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lbmk
