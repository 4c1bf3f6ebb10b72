// D2Q9 kernels (see lbm2d.h for the layout and the stage order).
#include "lbm2d.h"

namespace lbm2d {
namespace {

__device__ __forceinline__ double wgt(int i) { return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0); }

enum { GAS = 0, INERT = 1, CATALYTIC = 2 };
enum { UNIFORM = 0, WEIGHTED = 1, BOUNCEBACK = 2 };
enum { PASSIVE = 0, BARYCENTRIC = 1 };
enum { XPERIODIC = 0, XRESERVOIR = 1, XINFLOW = 2 };

__device__ __forceinline__ int wrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// second-order equilibrium of density r moving with (ux, uy)
__device__ __forceinline__ double feq(int i, double r, double ux, double uy) {
    const double cu = CX[i] * ux + CY[i] * uy, uu = ux * ux + uy * uy;
    return wgt(i) * r * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
}

__device__ __forceinline__ void moments(const double *f, int64_t n, int64_t node, double &r, double &jx,
                                        double &jy) {
    r = jx = jy = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double v = f[i * n + node];
        r += v;
        jx += CX[i] * v;
        jy += CY[i] * v;
    }
}

// Deterministic sum of NV values over a block of THREADS threads; thread 0
// writes them to out[0 .. NV).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *out) {
    __shared__ double sh[NV][THREADS];
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int w = THREADS / 2; w >= 1; w >>= 1) {
        if (int(threadIdx.x) < w)
#pragma unroll
            for (int k = 0; k < NV; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) out[k] = sh[k][0];
}

__global__ __launch_bounds__(THREADS) void k_init(Dev d, double rho0, double c0) {
    const int64_t node = int64_t(blockIdx.x) * THREADS + threadIdx.x;
    if (node >= d.n) return;
    const bool gas = d.vox[node] == GAS;
    for (int i = 0; i < Q; ++i) {
        d.fC[i * d.n + node] = gas ? feq(i, rho0, 0.0, 0.0) : 0.0;
        d.fR[i * d.n + node] = gas ? feq(i, c0, 0.0, 0.0) : 0.0;
        if (d.ph.product) d.fP[i * d.n + node] = 0.0;
        d.em[i * d.n + node] = 0.0;
        if (d.ph.product) d.emP[i * d.n + node] = 0.0;
    }
    d.acc[node] = 0.0;
    if (d.ph.product) d.accP[node] = 0.0;
}

// lattice masses of the initial state (partials as the stream writes them)
__global__ __launch_bounds__(THREADS) void k_mass(Dev d) {
    const int64_t node = int64_t(blockIdx.x) * THREADS + threadIdx.x;
    double v[NPS] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (node < d.n && d.vox[node] == GAS)
        for (int i = 0; i < Q; ++i) {
            v[0] += d.fC[i * d.n + node];
            v[1] += d.fR[i * d.n + node];
            if (d.ph.product) v[2] += d.fP[i * d.n + node];
        }
    block_sum<NPS>(v, d.part_s + int64_t(blockIdx.x) * NPS);
}

// Stage 1: BGK collision of every lattice at the gas nodes.
__global__ __launch_bounds__(THREADS) void k_collide(Dev d) {
    const int64_t node = int64_t(blockIdx.x) * THREADS + threadIdx.x;
    if (node >= d.n || d.vox[node] != GAS) return;
    const Params &P = d.ph;
    double rc, jcx, jcy, rr, jrx, jry, rp = 0.0, jpx = 0.0, jpy = 0.0;
    moments(d.fC, d.n, node, rc, jcx, jcy);
    moments(d.fR, d.n, node, rr, jrx, jry);
    if (P.product) moments(d.fP, d.n, node, rp, jpx, jpy);
    double ux, uy;
    if (P.coupling == BARYCENTRIC) {
        const double m = rc + rr + rp;
        ux = (jcx + jrx + jpx + 0.5 * P.force[0]) / m;
        uy = (jcy + jry + jpy + 0.5 * P.force[1]) / m;
    } else {
        ux = (jcx + 0.5 * P.force[0]) / rc;
        uy = (jcy + 0.5 * P.force[1]) / rc;
    }
    const double guo = 1.0 - 0.5 / P.tau_gas;
    for (int i = 0; i < Q; ++i) {
        const int64_t e = i * d.n + node;
        const double cu = CX[i] * ux + CY[i] * uy;
        const double src = guo * wgt(i) *
                           ((3.0 * (CX[i] - ux) + 9.0 * cu * CX[i]) * P.force[0] +
                            (3.0 * (CY[i] - uy) + 9.0 * cu * CY[i]) * P.force[1]);
        d.pC[e] = d.fC[e] - (d.fC[e] - feq(i, rc, ux, uy)) / P.tau_gas + src;
        d.pR[e] = d.fR[e] - (d.fR[e] - feq(i, rr, ux, uy)) / P.tau_species;
        if (P.product) d.pP[e] = d.fP[e] - (d.fP[e] - feq(i, rp, ux, uy)) / P.tau_species;
    }
}

// Stage 2: the sputtering condition at the catalytic nodes: In(k) over the
// active links (sources k - c_j that are gas nodes in the domain), E_i(k)
// along the reversed links, the running sums, and the arrivals of the step.
__global__ __launch_bounds__(THREADS) void k_interface(Dev d) {
    const int64_t node = int64_t(blockIdx.x) * THREADS + threadIdx.x;
    double v[NPI] = {0.0, 0.0};
    const uint32_t act = node < d.n && d.vox[node] == CATALYTIC ? d.mask[node] : 0u;
    if (act) {
        const Params &P = d.ph;
        const int x = int(node % d.nx), y = int(node / d.nx);
        double in = 0.0, in_p = 0.0, wsum = 0.0;
        int b = 0;
        for (int j = 1; j < Q; ++j) {
            if (!((act >> j) & 1u)) continue;
            const int64_t s = int64_t(wrap(y - CY[j], d.ny)) * d.nx + wrap(x - CX[j], d.nx);
            in += d.pR[j * d.n + s];
            if (P.product) in_p += d.pP[j * d.n + s];
            wsum += wgt(OPP[j]);
            ++b;
        }
        d.acc[node] += in;
        if (P.product) d.accP[node] += in_p;
        v[0] = in;
        v[1] = in_p;
        const double a_r = P.p * P.p_stick, a_p = 1.0 - P.p_stick_product;
        for (int j = 1; j < Q; ++j) {
            if (!((act >> j) & 1u)) continue;
            const int i = OPP[j];
            double e, ep;
            if (P.sputter == UNIFORM) {
                e = (1.0 - P.p_stick) * in / b;
                ep = (a_r * in + a_p * in_p) / b;
            } else if (P.sputter == WEIGHTED) {
                e = (1.0 - P.p_stick) * in * wgt(i) / wsum;
                ep = (a_r * in + a_p * in_p) * wgt(i) / wsum;
            } else {
                const int64_t s = int64_t(wrap(y - CY[j], d.ny)) * d.nx + wrap(x - CX[j], d.nx);
                e = (1.0 - P.p_stick) * d.pR[j * d.n + s];
                ep = a_r * d.pR[j * d.n + s] + (P.product ? a_p * d.pP[j * d.n + s] : 0.0);
            }
            d.em[i * d.n + node] = e;
            if (P.product) d.emP[i * d.n + node] = ep;
        }
    }
    block_sum<NPI>(v, d.part_i + int64_t(blockIdx.x) * NPI);
}

// Pull of one species into gas node (x, y): post-collision pst, emission em,
// inlet ghost values ghost[i] (species x-boundary reservoir or inflow:
// x = -1 is the ghost, x = nx a copy of plane nx - 1).
__device__ __forceinline__ double pull_species(const Dev &d, const double *pst, const double *em,
                                               const double (&ghost)[Q], int x, int y, int64_t node, int i,
                                               bool xper) {
    int sx = x - CX[i];
    const int sy = wrap(y - CY[i], d.ny);
    if (xper) sx = wrap(sx, d.nx);
    if (sx < 0) return ghost[i];
    if (sx >= d.nx) {
        const int64_t m = int64_t(sy) * d.nx + (d.nx - 1);
        return d.vox[m] == GAS ? pst[i * d.n + m] : pst[OPP[i] * d.n + node];
    }
    const int64_t s = int64_t(sy) * d.nx + sx;
    const uint8_t v = d.vox[s];
    return v == GAS ? pst[i * d.n + s] : (v == INERT ? pst[OPP[i] * d.n + node] : em[i * d.n + s]);
}

// Stage 3: streaming of every lattice into the gas nodes, the species that
// crossed the x-boundaries, and the lattice masses.
__global__ __launch_bounds__(THREADS) void k_stream(Dev d) {
    const int64_t node = int64_t(blockIdx.x) * THREADS + threadIdx.x;
    double v[NPS] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (node < d.n && d.vox[node] == GAS) {
        const Params &P = d.ph;
        const int x = int(node % d.nx), y = int(node / d.nx);
        // carrier: periodic in x, every solid reflects (a fraction sigma diffusely)
        double fc[Q], M = 0.0, W = 0.0;
        uint32_t solid = 0;
        for (int i = 0; i < Q; ++i) {
            const int64_t s = int64_t(wrap(y - CY[i], d.ny)) * d.nx + wrap(x - CX[i], d.nx);
            if (d.vox[s] == GAS) {
                fc[i] = d.pC[i * d.n + s];
            } else {
                fc[i] = d.pC[OPP[i] * d.n + node];
                M += fc[i];
                W += wgt(i);
                solid |= 1u << i;
            }
        }
        if (P.sigma != 0.0 && W > 0.0)
            for (int i = 0; i < Q; ++i)
                if ((solid >> i) & 1u) fc[i] = (1.0 - P.sigma) * fc[i] + P.sigma * wgt(i) * M / W;
        for (int i = 0; i < Q; ++i) {
            d.fC[i * d.n + node] = fc[i];
            v[0] += fc[i];
        }
        // inlet ghost of the reactant: the reservoir at rest, or (INFLOW) moving
        // with this node's carrier velocity
        double ghost[Q], none[Q];
        for (int i = 0; i < Q; ++i) {
            ghost[i] = wgt(i) * P.c_inlet;
            none[i] = 0.0;
        }
        if (P.species_x == XINFLOW && x == 0) {
            double r = 0.0, jx = 0.0, jy = 0.0;
            for (int i = 0; i < Q; ++i) {
                r += fc[i];
                jx += CX[i] * fc[i];
                jy += CY[i] * fc[i];
            }
            const double ux = (jx + 0.5 * P.force[0]) / r, uy = (jy + 0.5 * P.force[1]) / r;
            for (int i = 0; i < Q; ++i) ghost[i] = feq(i, P.c_inlet, ux, uy);
        }
        const bool xper = P.species_x == XPERIODIC;
        const bool first = !xper && x == 0, last = !xper && x == d.nx - 1;
        for (int i = 0; i < Q; ++i) {
            const double fr = pull_species(d, d.pR, d.em, ghost, x, y, node, i, xper);
            d.fR[i * d.n + node] = fr;
            v[1] += fr;
            if (first && CX[i] == 1) v[3] += fr;                    // pulled from the inlet ghost
            if (first && CX[i] == -1) v[4] += d.pR[i * d.n + node];  // left through the inlet face
            if (last && CX[i] == 1) v[5] += d.pR[i * d.n + node];   // sent to the outlet ghost
            if (last && CX[i] == -1) v[5] -= fr;                    // came back from it
            if (P.product) {
                const double fp = pull_species(d, d.pP, d.emP, none, x, y, node, i, xper);
                d.fP[i * d.n + node] = fp;
                v[2] += fp;
                if (first && CX[i] == -1) v[6] += d.pP[i * d.n + node];
                if (last && CX[i] == 1) v[7] += d.pP[i * d.n + node];
                if (last && CX[i] == -1) v[7] -= fp;
            }
        }
    }
    block_sum<NPS>(v, d.part_s + int64_t(blockIdx.x) * NPS);
}

// Stage 4 (one block): partial sums in block order, added to the totals.
// full = false after k_mass: only the masses are set.
__global__ __launch_bounds__(THREADS) void k_reduce(Dev d, int nb, bool full) {
    double v[NPI + NPS];
    for (int k = 0; k < NPI + NPS; ++k) v[k] = 0.0;
    for (int b = threadIdx.x; b < nb; b += THREADS) {
        if (full)
            for (int k = 0; k < NPI; ++k) v[k] += d.part_i[int64_t(b) * NPI + k];
        for (int k = 0; k < NPS; ++k) v[NPI + k] += d.part_s[int64_t(b) * NPS + k];
    }
    double out[NPI + NPS];
    block_sum<NPI + NPS>(v, out);
    if (threadIdx.x != 0) return;
    const Params &P = d.ph;
    double *t = d.tot;
    t[0] = out[NPI + 0];
    t[1] = out[NPI + 1];
    t[6] = out[NPI + 2];
    if (full) {
        t[2] += P.p * P.p_stick * out[0];
        t[3] += (1.0 - P.p) * P.p_stick * out[0];
        t[4] += out[NPI + 3];
        t[5] += out[NPI + 4] + out[NPI + 5];
        t[7] += P.p_stick_product * out[1];
        t[8] += out[NPI + 6];
        t[9] += out[NPI + 7];
    }
    bool bad = false;
    for (int k = 0; k < 10; ++k) bad |= !isfinite(t[k]);
    if (bad) t[10] = 1.0;
}

// Moments for the field outputs: rho_C, u (carrier velocity (j + F/2) / rho,
// or the barycentric one; component-major, u_z = 0), rho_R, rho_P; solid 0.
__global__ __launch_bounds__(THREADS) void k_fields(Dev d, double *rho, double *u, double *conc, double *rhoP) {
    const int64_t node = int64_t(blockIdx.x) * THREADS + threadIdx.x;
    if (node >= d.n) return;
    double rc = 0, jcx = 0, jcy = 0, rr = 0, jrx = 0, jry = 0, rp = 0, jpx = 0, jpy = 0, ux = 0, uy = 0;
    if (d.vox[node] == GAS) {
        moments(d.fC, d.n, node, rc, jcx, jcy);
        moments(d.fR, d.n, node, rr, jrx, jry);
        if (d.ph.product) moments(d.fP, d.n, node, rp, jpx, jpy);
        if (d.ph.coupling == BARYCENTRIC) {
            ux = (jcx + jrx + jpx + 0.5 * d.ph.force[0]) / (rc + rr + rp);
            uy = (jcy + jry + jpy + 0.5 * d.ph.force[1]) / (rc + rr + rp);
        } else {
            ux = (jcx + 0.5 * d.ph.force[0]) / rc;
            uy = (jcy + 0.5 * d.ph.force[1]) / rc;
        }
    }
    if (rho) rho[node] = rc;
    if (conc) conc[node] = rr;
    if (rhoP) rhoP[node] = rp;
    if (u) {
        u[node] = ux;
        u[d.n + node] = uy;
        u[2 * d.n + node] = 0.0;
    }
}

// Phi_P(x) = sum_y rho_P u_x, one thread per x, y ascending
__global__ __launch_bounds__(THREADS) void k_phi(Dev d, const double *rhoP, const double *u, double *phi) {
    const int x = int(blockIdx.x) * THREADS + int(threadIdx.x);
    if (x >= d.nx) return;
    double s = 0.0;
    for (int y = 0; y < d.ny; ++y) {
        const int64_t node = int64_t(y) * d.nx + x;
        s += rhoP[node] * u[node];
    }
    phi[x] = s;
}

}  // namespace

int blocks(int64_t n) { return int((n + THREADS - 1) / THREADS); }

hipError_t launch_init(const Dev &d, double rho0, double c0, hipStream_t s) {
    const int nb = blocks(d.n);
    hipLaunchKernelGGL(k_init, dim3(nb), dim3(THREADS), 0, s, d, rho0, c0);
    hipLaunchKernelGGL(k_mass, dim3(nb), dim3(THREADS), 0, s, d);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(THREADS), 0, s, d, nb, false);
    return hipGetLastError();
}

hipError_t launch_step(const Dev &d, hipStream_t s) {
    const int nb = blocks(d.n);
    hipLaunchKernelGGL(k_collide, dim3(nb), dim3(THREADS), 0, s, d);
    hipLaunchKernelGGL(k_interface, dim3(nb), dim3(THREADS), 0, s, d);
    hipLaunchKernelGGL(k_stream, dim3(nb), dim3(THREADS), 0, s, d);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(THREADS), 0, s, d, nb, true);
    return hipGetLastError();
}

hipError_t launch_fields(const Dev &d, double *rho, double *u, double *conc, double *rhoP, double *phi,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_fields, dim3(blocks(d.n)), dim3(THREADS), 0, s, d, rho, u, conc, rhoP);
    if (phi) hipLaunchKernelGGL(k_phi, dim3(blocks(d.nx)), dim3(THREADS), 0, s, d, rhoP, u, phi);
    return hipGetLastError();
}

}  // namespace lbm2d
