// HIP kernels of the reactive two-lattice lattice-Boltzmann step for gfx950.
//
// One time step (Falcucci et al., Appendix "Numerical Method"):
//   k_interface  sputtering boundary condition: every catalytic node k sums
//                the reactant arriving along its active links,
//                In(k) = sum_j f*_j(k - c_j) (first line of the sputtering
//                equations), accumulates it and stores the re-emission
//                (1 - p_S^R) In(k) scale(k);
//   k_xflux      species crossing the x reservoir planes (bookkeeping);
//   k_sweep      fused pull-streaming + BGK collision of both lattices,
//                Eq. LBE with the second-order equilibrium, Guo body force on
//                the carrier, halfway bounce-back at solid links, the reactive
//                pull at catalytic sources and the reservoir ghosts;
//   k_reduce     fixed-order FP64 totals.
//
// Storage: populations of gas nodes only, structure of arrays
// f[lattice][direction][gas node] in (z, y, x) order, as the normalised
// deviation h_i = f_i / w_i - rho_ref (rho_ref = rho0 for the carrier, c_ref
// for the reactant).  A wavefront owns one 64-voxel chunk of an x-row; lanes
// on solid voxels idle.  A gas neighbour's storage index is its chunk base
// plus a popcount of the chunk's gas bits, so no per-node neighbour table is
// read: the 32-byte chunk records of the nine source rows are scalar loads.
// Memory traffic is therefore close to 2 x 38 populations per gas node.

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "lbm_internal.h"

namespace lbmk {
namespace {

// Row offset slot of (cy, cz): 9 source rows.
__host__ __device__ constexpr int row_slot(int cy, int cz) { return (cy + 1) * 3 + (cz + 1); }

// ------------------------------------------------------------ storage --
template <int ST>
struct Store;
template <>
struct Store<ST_F32> {
    using S = float;
    using T = float;
    __device__ static T ld(const S *p) { return *p; }
    __device__ static void st(S *p, T v) { *p = v; }
};
template <>
struct Store<ST_F16> {
    using S = _Float16;
    using T = float;
    __device__ static T ld(const S *p) { return static_cast<float>(*p); }
    __device__ static void st(S *p, T v) { *p = static_cast<_Float16>(v); }  // round to nearest even
};
template <>
struct Store<ST_BF16> {
    using S = uint16_t;
    using T = float;
    __device__ static T ld(const S *p) { return __uint_as_float(uint32_t(*p) << 16); }
    __device__ static void st(S *p, T v) {
        uint32_t u = __float_as_uint(v);
        if ((u & 0x7fffffffu) > 0x7f800000u) {
            *p = uint16_t((u >> 16) | 0x40u);  // quiet NaN stays NaN
            return;
        }
        u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
        *p = uint16_t(u >> 16);
    }
};
template <>
struct Store<ST_F64> {
    using S = double;
    using T = double;
    __device__ static T ld(const S *p) { return *p; }
    __device__ static void st(S *p, T v) { *p = v; }
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
    T h0c, h0r;       // initial state, normalised: rho0 - rho_ref, c0 - c_ref
    int32_t sputter, coupling, species_x;
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
    k.h0c = T(p.rho0 - p.rho_ref);
    k.h0r = T(p.c0 - p.c_ref);
    k.sputter = p.sputter;
    k.coupling = p.coupling;
    k.species_x = p.species_x;
    return k;
}

// ------------------------------------------------------------ helpers --
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
        for (int k = 0; k < NV; ++k) out[k] = ((sh[0][k] + sh[1][k]) + sh[2][k]) + sh[3][k];
}

// Source of a pull along a direction with x-component cx, seen from this
// lane, in the source row described by I.  `below` counts the gas bits of
// I.fluid below this lane.
struct Src {
    bool fluid, cat;
    uint32_t rank;
};

__device__ __forceinline__ Src source_in_row(const ChunkInfo &I, uint32_t below, int lane, int cx, bool last_x) {
    Src s;
    if (cx == 0) {
        s.fluid = (I.fluid >> lane) & 1u;
        s.cat = (I.cat >> lane) & 1u;
        s.rank = I.base + below;
    } else if (cx == 1) {  // source x - 1
        if (lane > 0) {
            const uint32_t b = uint32_t(I.fluid >> (lane - 1)) & 1u;
            s.fluid = b;
            s.cat = (I.cat >> (lane - 1)) & 1u;
            s.rank = I.base + below - b;
        } else {
            s.fluid = I.edge & 1u;
            s.cat = I.edge & 2u;
            s.rank = I.prev_rank;
        }
    } else {  // cx == -1, source x + 1
        if (lane < 63 && !last_x) {
            s.fluid = (I.fluid >> (lane + 1)) & 1u;
            s.cat = (I.cat >> (lane + 1)) & 1u;
            s.rank = I.base + below + (uint32_t(I.fluid >> lane) & 1u);
        } else {
            s.fluid = I.edge & 4u;
            s.cat = I.edge & 8u;
            s.rank = I.next_rank;
        }
    }
    return s;
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
    // contiguous range of rows so neighbouring rows share its L2.
    const int per = nb >> 3;
    if ((nb & 7) != 0 || per == 0) return b;
    return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ WaveUnit locate(const Geometry &g) {
    WaveUnit u;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int64_t unit = int64_t(xcd_block(int(blockIdx.x), int(gridDim.x))) * 4 + wave;
    const int64_t units = int64_t(g.ny) * g.nz * g.W;
    u.valid = unit < units;
    const int64_t un = u.valid ? unit : 0;
    u.row = __builtin_amdgcn_readfirstlane(int(un / g.W));
    u.chunk = __builtin_amdgcn_readfirstlane(int(un - int64_t(u.row) * g.W));
    u.y = u.row % g.ny;
    u.z = u.row / g.ny;
    u.lane = int(threadIdx.x & 63);
    u.x = u.chunk * 64 + u.lane;
    const ChunkInfo &I = g.chunks[int64_t(u.row) * g.W + u.chunk];
    const uint64_t fl = I.fluid;
    u.active = u.valid && u.x < g.nx && ((fl >> u.lane) & 1u);
    u.idx = I.base + bits_below_lane(fl);
    return u;
}

// Pull both lattices into registers: hC[i], hR[i] are the normalised
// populations of this node after streaming (the pre-collision state).
template <int ST>
__device__ __forceinline__ void pull(const Geometry &g, const PhysK<typename Store<ST>::T> &ph,
                                     const typename Store<ST>::S *__restrict__ fin,
                                     const typename Store<ST>::T *__restrict__ emit, const WaveUnit &u,
                                     typename Store<ST>::T (&hC)[19], typename Store<ST>::T (&hR)[19]) {
    using T = typename Store<ST>::T;
    using S = typename Store<ST>::S;
    const int64_t nfp = g.nfp;
    const S *finR = fin + 19 * nfp;
    const bool reservoir = ph.species_x == XB_RESERVOIR;
    const bool first_x = u.x == 0, last_x = u.x == g.nx - 1;

    // the nine source rows (uniform per wave)
    ChunkInfo rows[9];
    uint32_t below[9];
#pragma unroll
    for (int cy = -1; cy <= 1; ++cy)
#pragma unroll
        for (int cz = -1; cz <= 1; ++cz) {
            int ys = u.y - cy, zs = u.z - cz;
            ys = ys < 0 ? ys + g.ny : (ys >= g.ny ? ys - g.ny : ys);
            zs = zs < 0 ? zs + g.nz : (zs >= g.nz ? zs - g.nz : zs);
            const int r = __builtin_amdgcn_readfirstlane(zs * g.ny + ys);
            rows[row_slot(cy, cz)] = g.chunks[int64_t(r) * g.W + u.chunk];
            below[row_slot(cy, cz)] = bits_below_lane(rows[row_slot(cy, cz)].fluid);
        }

    hC[0] = Store<ST>::ld(fin + u.idx);
    hR[0] = Store<ST>::ld(finR + u.idx);
#pragma unroll
    for (int i = 1; i < 19; ++i) {
        const int slot = row_slot(CY[i], CZ[i]);
        const ChunkInfo &I = rows[slot];
        const Src s = source_in_row(I, below[slot], u.lane, CX[i], last_x);
        // carrier: periodic in x, every solid reflects
        const S *ac = s.fluid ? fin + i * nfp + s.rank : fin + opp(i) * nfp + u.idx;
        hC[i] = Store<ST>::ld(ac);
        // reactant
        bool sf = s.fluid, sc = s.cat;
        uint32_t rank = s.rank;
        bool inlet = false;
        if (reservoir && CX[i] == 1 && first_x) {
            inlet = true;
        } else if (reservoir && CX[i] == -1 && last_x) {
            // outlet ghost: copy of plane nx - 1 at the source row
            sf = (I.fluid >> u.lane) & 1u;
            sc = false;
            rank = I.base + below[slot];
        }
        const bool cat = !inlet && !sf && sc;
        const bool bb_cat = cat && ph.sputter == SP_BOUNCEBACK;
        T v = ph.h_inlet;
        if (!inlet && (!cat || bb_cat)) {
            const S *ar = sf ? finR + i * nfp + rank : finR + opp(i) * nfp + u.idx;
            v = Store<ST>::ld(ar);
            if (bb_cat) v = ph.keep * (v + ph.cref) - ph.cref;
        }
        if (cat && !bb_cat) {
            int xs = u.x - CX[i];
            xs = xs < 0 ? xs + g.nx : (xs >= g.nx ? xs - g.nx : xs);
            int ys = u.y - CY[i], zs = u.z - CZ[i];
            ys = ys < 0 ? ys + g.ny : (ys >= g.ny ? ys - g.ny : ys);
            zs = zs < 0 ? zs + g.nz : (zs >= g.nz ? zs - g.nz : zs);
            const T e = emit[(int64_t(zs) * g.ny + ys) * g.nx + xs];
            v = (ph.sputter == SP_UNIFORM ? e * inv_wgt<T>(i) : e) - ph.cref;
        }
        hR[i] = v;
    }
}

// Moments of both lattices and the equilibrium velocity.
template <typename T>
struct Mom {
    T dc, rc, dr, rr;  // density deviations and densities
    T ux, uy, uz;
};

template <typename T>
__device__ __forceinline__ Mom<T> moments(const PhysK<T> &ph, const T (&hC)[19], const T (&hR)[19]) {
    Mom<T> m;
    T dc = 0, jx = 0, jy = 0, jz = 0, dr = 0, rx = 0, ry = 0, rz = 0;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const T a = wgt<T>(i) * hC[i], b = wgt<T>(i) * hR[i];
        dc += a;
        dr += b;
        if (CX[i]) { jx += CX[i] * a; rx += CX[i] * b; }
        if (CY[i]) { jy += CY[i] * a; ry += CY[i] * b; }
        if (CZ[i]) { jz += CZ[i] * a; rz += CZ[i] * b; }
    }
    m.dc = dc;
    m.dr = dr;
    m.rc = ph.rref + dc;
    m.rr = ph.cref + dr;
    if (ph.coupling == CP_BARYCENTRIC) {
        const T inv = T(1) / (m.rc + m.rr);
        m.ux = (jx + rx + T(0.5) * ph.fx) * inv;
        m.uy = (jy + ry + T(0.5) * ph.fy) * inv;
        m.uz = (jz + rz + T(0.5) * ph.fz) * inv;
    } else {
        const T inv = T(1) / m.rc;
        m.ux = (jx + T(0.5) * ph.fx) * inv;
        m.uy = (jy + T(0.5) * ph.fy) * inv;
        m.uz = (jz + T(0.5) * ph.fz) * inv;
    }
    return m;
}

// BGK collision in normalised form: h* = h - omega (h - heq) (+ Guo / w_i on
// the carrier), heq_i = (rho - rho_ref) + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u).
template <typename T>
__device__ __forceinline__ void collide(const PhysK<T> &ph, const Mom<T> &m, T (&hC)[19], T (&hR)[19]) {
    const T uu = m.ux * m.ux + m.uy * m.uy + m.uz * m.uz;
    const T uf = m.ux * ph.fx + m.uy * ph.fy + m.uz * ph.fz;
    const T base_c = m.dc - T(1.5) * m.rc * uu, base_r = m.dr - T(1.5) * m.rr * uu;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const T cu = T(CX[i]) * m.ux + T(CY[i]) * m.uy + T(CZ[i]) * m.uz;
        const T cf = T(CX[i]) * ph.fx + T(CY[i]) * ph.fy + T(CZ[i]) * ph.fz;
        const T poly = T(3) * cu + T(4.5) * cu * cu;
        const T eqc = base_c + m.rc * poly;
        const T eqr = base_r + m.rr * poly;
        const T src = ph.guo * (T(3) * (cf - uf) + T(9) * cu * cf);
        hC[i] = hC[i] - ph.om_c * (hC[i] - eqc) + src;
        hR[i] = hR[i] - ph.om_r * (hR[i] - eqr);
    }
}

// ------------------------------------------------------------ kernels --

template <int ST>
__global__ __launch_bounds__(256) void k_sweep(Geometry g, PhysK<typename Store<ST>::T> ph,
                                                const typename Store<ST>::S *__restrict__ fin,
                                                typename Store<ST>::S *__restrict__ fout,
                                                const typename Store<ST>::T *__restrict__ emit,
                                                double *__restrict__ part) {
    using T = typename Store<ST>::T;
    const WaveUnit u = locate(g);
    double acc[2] = {0.0, 0.0};
    if (u.active) {
        T hC[19], hR[19];
        pull<ST>(g, ph, fin, emit, u, hC, hR);
        const Mom<T> m = moments(ph, hC, hR);
        acc[0] = double(m.rc);
        acc[1] = double(m.rr);
        collide(ph, m, hC, hR);
        const int64_t nfp = g.nfp;
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            Store<ST>::st(fout + i * nfp + u.idx, hC[i]);
            Store<ST>::st(fout + (19 + i) * nfp + u.idx, hR[i]);
        }
    }
    block_sum<2>(acc, part + int64_t(blockIdx.x) * 2);
}

template <int ST, bool LOCAL, typename OUT>
__global__ __launch_bounds__(256) void k_fields(Geometry g, PhysK<typename Store<ST>::T> ph,
                                                 const typename Store<ST>::S *__restrict__ fin,
                                                 const typename Store<ST>::T *__restrict__ emit, OUT *rho, OUT *vel,
                                                 OUT *conc) {
    using T = typename Store<ST>::T;
    const WaveUnit u = locate(g);
    if (!u.valid || u.x >= g.nx) return;
    T r = 0, ux = 0, uy = 0, uz = 0, c = 0;
    if (u.active) {
        T hC[19], hR[19];
        if (LOCAL) {
#pragma unroll
            for (int i = 0; i < 19; ++i) {
                hC[i] = Store<ST>::ld(fin + i * g.nfp + u.idx);
                hR[i] = Store<ST>::ld(fin + (19 + i) * g.nfp + u.idx);
            }
        } else {
            pull<ST>(g, ph, fin, emit, u, hC, hR);
        }
        const Mom<T> m = moments(ph, hC, hR);
        r = m.rc;
        c = m.rr;
        ux = m.ux;
        uy = m.uy;
        uz = m.uz;
    }
    const int64_t n = int64_t(g.nx) * g.ny * g.nz;
    const int64_t v = int64_t(u.row) * g.nx + u.x;
    if (rho) rho[v] = OUT(r);
    if (conc) conc[v] = OUT(c);
    if (vel) {
        vel[v] = OUT(ux);
        vel[n + v] = OUT(uy);
        vel[2 * n + v] = OUT(uz);
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
    if (n >= g.nfluid) return;
    T hC[19], hR[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        hC[i] = ph.h0c;
        hR[i] = ph.h0r;
        Store<ST>::st(pre + i * g.nfp + n, hC[i]);
        Store<ST>::st(pre + (19 + i) * g.nfp + n, hR[i]);
    }
    const Mom<T> m = moments(ph, hC, hR);
    collide(ph, m, hC, hR);
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        Store<ST>::st(post + i * g.nfp + n, hC[i]);
        Store<ST>::st(post + (19 + i) * g.nfp + n, hR[i]);
    }
}

__device__ __forceinline__ uint32_t rank_of(const Geometry &g, int row, int x, bool *fluid) {
    const ChunkInfo &I = g.chunks[int64_t(row) * g.W + (x >> 6)];
    const int b = x & 63;
    *fluid = (I.fluid >> b) & 1u;
    const uint64_t below = b ? (I.fluid & (~0ull >> (64 - b))) : 0ull;
    return I.base + uint32_t(__popcll(below));
}

// Sputtering gather: In(k) over the active links of each interface node.
template <int ST>
__global__ __launch_bounds__(256) void k_interface(Geometry g, PhysK<typename Store<ST>::T> ph, Interface it,
                                                    const typename Store<ST>::S *__restrict__ fin,
                                                    typename Store<ST>::T *__restrict__ emit,
                                                    double *__restrict__ part) {
    using T = typename Store<ST>::T;
    using S = typename Store<ST>::S;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    double arrived[1] = {0.0};
    if (k < it.n) {
        const uint32_t v = it.vox[k];
        const uint32_t mask = it.mask[k];
        const int x = int(v % uint32_t(g.nx));
        const int row = int(v / uint32_t(g.nx));
        const int y = row % g.ny, z = row / g.ny;
        const S *finR = fin + 19 * g.nfp;
        double in = 0.0;
#pragma unroll
        for (int j = 1; j < 19; ++j) {
            if (mask & (1u << j)) {
                int xs = x - CX[j], ys = y - CY[j], zs = z - CZ[j];
                xs = xs < 0 ? xs + g.nx : (xs >= g.nx ? xs - g.nx : xs);
                ys = ys < 0 ? ys + g.ny : (ys >= g.ny ? ys - g.ny : ys);
                zs = zs < 0 ? zs + g.nz : (zs >= g.nz ? zs - g.nz : zs);
                bool fl;
                const uint32_t r = rank_of(g, zs * g.ny + ys, xs, &fl);
                const T h = Store<ST>::ld(finR + j * g.nfp + r);
                in += double(wgt<T>(j) * (h + ph.cref));
            }
        }
        it.acc[k] += in;
        if (ph.sputter != SP_BOUNCEBACK) emit[v] = T(double(ph.keep) * in * it.scale[k]);
        arrived[0] = in;
    }
    block_sum<1>(arrived, part + blockIdx.x);
}

// Species crossing the reservoir planes during the coming streaming: influx
// pulled from the inlet ghost, and what leaves through x = -1 and x = nx net
// of what the outlet ghost returns.  One lane per x-row.
template <int ST>
__global__ __launch_bounds__(256) void k_xflux(Geometry g, PhysK<typename Store<ST>::T> ph, double c_inlet,
                                                const typename Store<ST>::S *__restrict__ fin,
                                                double *__restrict__ part) {
    using T = typename Store<ST>::T;
    using S = typename Store<ST>::S;
    const int64_t rows = int64_t(g.ny) * g.nz;
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    double acc[2] = {0.0, 0.0};
    if (r < rows) {
        const S *finR = fin + 19 * g.nfp;
        const int y = int(r % g.ny), z = int(r / g.ny);
        bool fl;
        const uint32_t r0 = rank_of(g, int(r), 0, &fl);
        if (fl) {
#pragma unroll
            for (int i = 1; i < 19; ++i) {
                if (CX[i] == 1) acc[0] += double(wgt<T>(i)) * c_inlet;
                if (CX[i] == -1) acc[1] += double(wgt<T>(i) * (Store<ST>::ld(finR + i * g.nfp + r0) + ph.cref));
            }
        }
        const uint32_t r1 = rank_of(g, int(r), g.nx - 1, &fl);
        if (fl) {
#pragma unroll
            for (int i = 1; i < 19; ++i) {
                if (CX[i] == 1) acc[1] += double(wgt<T>(i) * (Store<ST>::ld(finR + i * g.nfp + r1) + ph.cref));
                if (CX[i] == -1) {
                    int ys = y - CY[i], zs = z - CZ[i];
                    ys = ys < 0 ? ys + g.ny : (ys >= g.ny ? ys - g.ny : ys);
                    zs = zs < 0 ? zs + g.nz : (zs >= g.nz ? zs - g.nz : zs);
                    bool mf;
                    const uint32_t rm = rank_of(g, zs * g.ny + ys, g.nx - 1, &mf);
                    const T h = mf ? Store<ST>::ld(finR + i * g.nfp + rm) : Store<ST>::ld(finR + opp(i) * g.nfp + r1);
                    acc[1] -= double(wgt<T>(i) * (h + ph.cref));
                }
            }
        }
    }
    block_sum<2>(acc, part + int64_t(blockIdx.x) * 2);
}

// Fixed-order sum of column `col` of a row-major [n][ncol] partial array.
__device__ double column_sum(const double *p, int64_t n, int ncol, int col) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += blockDim.x) s += p[r * ncol + col];
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

__global__ __launch_bounds__(256) void k_reduce(const double *ps, int64_t ns, const double *pi, int64_t ni,
                                                 const double *pf, int64_t nf, double p, double p_stick,
                                                 DevTotals *tot) {
    const double mc = column_sum(ps, ns, 2, 0);
    const double mr = column_sum(ps, ns, 2, 1);
    const double in = ni ? column_sum(pi, ni, 1, 0) : 0.0;
    const double fin = nf ? column_sum(pf, nf, 2, 0) : 0.0;
    const double fout = nf ? column_sum(pf, nf, 2, 1) : 0.0;
    if (threadIdx.x == 0) {
        tot->mass_gas = mc;
        tot->mass_species = mr;
        tot->converted += p * p_stick * in;
        tot->lost += (1.0 - p) * p_stick * in;
        tot->influx += fin;
        tot->outflux += fout;
        tot->step += 1;
        const double all = mc + mr + in + fin + fout;
        if (!(all - all == 0.0)) tot->nonfinite = 1;
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

int64_t sweep_blocks(const Geometry &g) { return (int64_t(g.ny) * g.nz * g.W + 3) / 4; }
int64_t interface_blocks(int64_t n) { return n > 0 ? (n + 255) / 256 : 0; }
int64_t xflux_blocks(const Geometry &g) { return (int64_t(g.ny) * g.nz + 255) / 256; }

hipError_t launch_init(const Geometry &g, const Physics &ph, void *pre, void *post, hipStream_t s) {
    return dispatch(ph.storage, [&](auto st) {
        constexpr int ST = decltype(st)::value;
        using SS = typename Store<ST>::S;
        using T = typename Store<ST>::T;
        const int64_t blocks = (g.nfluid + 255) / 256;
        if (blocks == 0) return hipSuccess;
        hipLaunchKernelGGL(k_init<ST>, dim3(unsigned(blocks)), dim3(256), 0, s, g, to_kernel<T>(ph),
                           static_cast<SS *>(pre), static_cast<SS *>(post));
        return hipGetLastError();
    });
}

hipError_t launch_interface(const Geometry &g, const Physics &ph, const Interface &it, const void *fin, void *emit,
                            double *part, int64_t blocks, hipStream_t s) {
    if (blocks == 0) return hipSuccess;
    return dispatch(ph.storage, [&](auto st) {
        constexpr int ST = decltype(st)::value;
        using SS = typename Store<ST>::S;
        using T = typename Store<ST>::T;
        hipLaunchKernelGGL(k_interface<ST>, dim3(unsigned(blocks)), dim3(256), 0, s, g, to_kernel<T>(ph), it,
                           static_cast<const SS *>(fin), static_cast<T *>(emit), part);
        return hipGetLastError();
    });
}

hipError_t launch_xflux(const Geometry &g, const Physics &ph, const void *fin, double *part, int64_t blocks,
                        hipStream_t s) {
    if (blocks == 0) return hipSuccess;
    return dispatch(ph.storage, [&](auto st) {
        constexpr int ST = decltype(st)::value;
        using SS = typename Store<ST>::S;
        using T = typename Store<ST>::T;
        hipLaunchKernelGGL(k_xflux<ST>, dim3(unsigned(blocks)), dim3(256), 0, s, g, to_kernel<T>(ph), ph.c_inlet,
                           static_cast<const SS *>(fin), part);
        return hipGetLastError();
    });
}

hipError_t launch_sweep(const Geometry &g, const Physics &ph, const void *fin, void *fout, const void *emit,
                        double *part, hipStream_t s) {
    return dispatch(ph.storage, [&](auto st) {
        constexpr int ST = decltype(st)::value;
        using SS = typename Store<ST>::S;
        using T = typename Store<ST>::T;
        hipLaunchKernelGGL(k_sweep<ST>, dim3(unsigned(sweep_blocks(g))), dim3(256), 0, s, g, to_kernel<T>(ph),
                           static_cast<const SS *>(fin), static_cast<SS *>(fout), static_cast<const T *>(emit), part);
        return hipGetLastError();
    });
}

hipError_t launch_fields(const Geometry &g, const Physics &ph, const void *fin, const void *emit, int mode, void *rho,
                         void *u, void *conc, bool out_f64, hipStream_t s) {
    return dispatch(ph.storage, [&](auto st) {
        constexpr int ST = decltype(st)::value;
        using SS = typename Store<ST>::S;
        using T = typename Store<ST>::T;
        const dim3 grid(unsigned(sweep_blocks(g))), block(256);
        const SS *f = static_cast<const SS *>(fin);
        const T *e = static_cast<const T *>(emit);
        const PhysK<T> k = to_kernel<T>(ph);
        if (out_f64) {
            double *a = static_cast<double *>(rho), *b = static_cast<double *>(u), *c = static_cast<double *>(conc);
            if (mode == 2)
                hipLaunchKernelGGL((k_fields<ST, true, double>), grid, block, 0, s, g, k, f, e, a, b, c);
            else
                hipLaunchKernelGGL((k_fields<ST, false, double>), grid, block, 0, s, g, k, f, e, a, b, c);
        } else {
            float *a = static_cast<float *>(rho), *b = static_cast<float *>(u), *c = static_cast<float *>(conc);
            if (mode == 2)
                hipLaunchKernelGGL((k_fields<ST, true, float>), grid, block, 0, s, g, k, f, e, a, b, c);
            else
                hipLaunchKernelGGL((k_fields<ST, false, float>), grid, block, 0, s, g, k, f, e, a, b, c);
        }
        return hipGetLastError();
    });
}

hipError_t launch_reduce(const double *part_sweep, int64_t n_sweep, const double *part_iface, int64_t n_iface,
                         const double *part_flux, int64_t n_flux, double p, double p_stick, DevTotals *tot,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, part_sweep, n_sweep, part_iface, n_iface, part_flux,
                       n_flux, p, p_stick, tot);
    return hipGetLastError();
}

}  // namespace lbmk
