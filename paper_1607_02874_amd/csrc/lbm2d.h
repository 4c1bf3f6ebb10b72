// The D2Q9 path: the paper's own lattice (Appendix "Numerical Method",
// Fig. A1) on one plane, for the 2-D reactor and the Leveque channel.
// Internal to the library (lbm_api.cpp dispatches the public entry points to
// it for contexts created with lbm_bc.lattice = LBM_LATTICE_D2Q9).
//
// Populations are FP64, direction-major over every node of the nx x ny
// plane (element i n + node, node = y nx + x, solid nodes unused).  One step
// runs the method in the order of its definition, one kernel per stage:
//   collide    BGK of every lattice (Guo forcing on the carrier) -> post
//   interface  In(k) of every catalytic node from the post-collision
//              reactant (and product) populations arriving along its active
//              links, the re-emission E_i(k), the running sum of In(k)
//   stream     pull of every lattice into the gas nodes (bounce-back,
//              emission at catalytic sources, inlet and outlet ghosts), the
//              species crossing the x-boundaries, the lattice masses
//   reduce     one block: the per-block partial sums in a fixed order, added
//              to the totals
// Every node is written by one thread and every sum has a fixed order, so
// results do not depend on the launch or the run.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbm2d {

constexpr int Q = 9;
// D2Q9 velocity set, numbered counter-clockwise: rest, the four axis links
// (w = 1/9), the four diagonals (w = 1/36); cs^2 = 1/3.
constexpr int CX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int CY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int OPP[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
constexpr int THREADS = 256;
// per-block partial sums: interface (arrived R, arrived P), stream (masses of
// C, R, P; influx, out through the inlet face, net out through the outlet
// face, the same two for P)
constexpr int NPI = 2, NPS = 8;
// device totals: mass C, mass R, converted, lost, influx, outflux,
// mass P, lost P, P out inlet, P out outlet, nonfinite flag
constexpr int NTOT = 11;

struct Params {
    double tau_gas, tau_species;
    double p, p_stick, p_stick_product;
    double c_inlet;
    double force[2];
    double sigma;  // diffuse fraction of the carrier wall
    int32_t sputter, coupling, species_x, product;
};

struct Dev {
    int32_t nx, ny;
    int64_t n;
    const uint8_t *vox;    // 0 gas, 1 inert, 2 catalytic
    const uint16_t *mask;  // per node: active links j (bit j) of a catalytic node
    double *fC, *fR, *fP;  // pre-collision [Q][n]
    double *pC, *pR, *pP;  // post-collision [Q][n]
    double *em, *emP;      // emission of catalytic nodes [Q][n]
    double *acc, *accP;    // per node: sum_t In(k, t), sum_t In_P(k, t)
    double *part_i, *part_s;  // per-block partials
    double *tot;           // NTOT totals
    Params ph;
};

hipError_t launch_init(const Dev &d, double rho0, double c0, hipStream_t s);
hipError_t launch_step(const Dev &d, hipStream_t s);
hipError_t launch_fields(const Dev &d, double *rho, double *u, double *conc, double *rhoP, double *phi,
                         hipStream_t s);
int blocks(int64_t n);

}  // namespace lbm2d
