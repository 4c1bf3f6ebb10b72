// Internal interface between the C-ABI host code (lbm_api.cpp) and the HIP
// kernels (lbm_kernels.hip).  Not installed, not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbmk {

// D3Q19 velocities in the library's numbering: 0 rest; 1..9 one of each
// velocity pair; 10..18 their negatives, so opp(i) = i + 9 (i <= 9) or i - 9.
// Weights: 1/3 (rest), 1/18 (axis), 1/36 (face diagonal).
constexpr int CX[19] = {0, 1, 0, 0, 1, 1, 1, 1, 0, 0, -1, 0, 0, -1, -1, -1, -1, 0, 0};
constexpr int CY[19] = {0, 0, 1, 0, 1, -1, 0, 0, 1, 1, 0, -1, 0, -1, 1, 0, 0, -1, -1};
constexpr int CZ[19] = {0, 0, 0, 1, 0, 0, 1, -1, 1, -1, 0, 0, -1, 0, 0, -1, 1, -1, 1};

__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : (i <= 9 ? i + 9 : i - 9); }

template <typename T>
__host__ __device__ constexpr T wgt(int i) {
    return i == 0 ? T(1) / T(3) : ((CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i]) == 1 ? T(1) / T(18) : T(1) / T(36));
}

template <typename T>
__host__ __device__ constexpr T inv_wgt(int i) {
    return i == 0 ? T(3) : ((CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i]) == 1 ? T(18) : T(36));
}

// One 64-voxel segment of an x-row.  The populations of gas nodes are stored
// compactly (gas nodes only, in (z, y, x) order), so a gas node's storage
// index is base + (number of gas bits below it in this chunk).
struct ChunkInfo {
    uint64_t fluid;   // bit b: voxel x = 64 c + b (< nx) is gas
    uint64_t cat;     // bit b: voxel is an interface node (catalytic, >= 1 active link)
    uint32_t base;    // storage index of the first gas voxel of the chunk
    uint32_t ibase;   // interface index of the first interface voxel of the chunk
    uint32_t prev;    // periodic left neighbour x = 64 c - 1: NB_GAS | storage index, NB_CAT | interface index, or 0
    uint32_t next;    // periodic right neighbour (x = 64 c + 64, or 0 after the last chunk), same encoding
};
// Neighbour-field flags; indices stay below 2^30 (checked at create).
constexpr uint32_t NB_GAS = 1u << 31, NB_CAT = 1u << 30, NB_IDX = NB_CAT - 1u;
static_assert(sizeof(ChunkInfo) == 32, "ChunkInfo must stay 32 bytes (one scalar load)");

enum { ST_F32 = 0, ST_F16 = 1, ST_BF16 = 2, ST_F64 = 3 };
enum { SP_UNIFORM = 0, SP_WEIGHTED = 1, SP_BOUNCEBACK = 2, SP_STOCHASTIC = 3 };
// STOCHASTIC keeps one In and one emission slot per exit direction of each
// interface node, direction-major: slot (e - 1) * n_interface + k for exit
// direction e, so lanes that pull from neighbouring interface nodes along
// one direction read neighbouring slots.
constexpr int NSLOT = 18;
enum { CP_PASSIVE = 0, CP_BARYCENTRIC = 1 };
enum { ROUND_NEAREST = 0, ROUND_STOCHASTIC = 1 };
enum { XB_PERIODIC = 0, XB_RESERVOIR = 1, XB_INFLOW = 2 };

// Slots of the per-step partial sums (FP64).  The sweep writes four per
// block (carrier mass, reactant mass, influx, outflux), the interface kernel
// one (arrivals In).  With the product lattice the sweep adds three per
// block (product mass, product leaving through the inlet face and through the
// outlet face) and the interface kernel one (product arrivals In_P).
enum {
    PART_MASS_C = 0, PART_MASS_R = 1, PART_IN = 2, PART_INFLUX = 3, PART_OUTFLUX = 4,
    PART_MASS_P = 5, PART_IN_P = 6, PART_POUT_IN = 7, PART_POUT_OUT = 8, NPART = 9
};
constexpr int NPART_BASE = 5;  // the slots without the product lattice

// Device totals: step-cumulative FP64 values and the non-finite flag.
struct DevTotals {
    double mass_gas, mass_species, converted, lost, influx, outflux;
    double mass_product, lost_product, product_out_inlet, product_out_outlet;
    int64_t step;
    int32_t nonfinite;
    int32_t pad;
};

struct Geometry {
    const ChunkInfo *chunks;  // rows * W records, row = z * ny + y
    const uint32_t *order;    // sweep traversal: per wave y | z << 12 | chunk << 24
    unsigned long long *inacc;  // per interface node: In(k) of the sweep in progress, fixed point (see Interface)
    int32_t nx, ny, nz, W;    // W = ceil(nx / 64)
    uint32_t units;           // ny * nz * W waves
    uint32_t niface;          // interface nodes (stride of the STOCHASTIC slot arrays)
    int64_t nfp;              // elements per direction in a population buffer
    int64_t nfluid;
    // Node-compact sweep (one lane per gas node, 64 consecutive storage
    // indices per wave); null when the lattice is too large for `pos`.
    const uint32_t *pos;      // per gas node: x | y << 12 | z << 22
    const uint32_t *worder;   // launch order of the 64-node waves
    const uint32_t *wunits;   // per wave: first (row, chunk) unit | units spanned << 26
    uint32_t nwaves;          // ceil(nfluid / 64)
    // Population layout: element (node n, slot s) of a population array
    // (pairs, or single product populations) is s lay_ss + (n >> 6) lay_bs +
    // (n & 63).  Blocked: lay_ss = 64, lay_bs = 19 * 64 (the 19 slots of 64
    // consecutive nodes form one contiguous block); slot-major: lay_ss = nfp,
    // lay_bs = 64 (element n of slot s at s nfp + n).
    uint32_t lay_ss, lay_bs;
    int32_t pad2;
    // 1 / W and 1 / ny: the compact sweep splits unit indices u = row W +
    // chunk and rows = z ny + y as trunc((n + 1/2) / d) in FP64, exact for
    // n < 2^26 and d <= 2^12.
    double inv_W, inv_ny;
    // interface list (voxel index and active-link mask per interface node),
    // read by the STOCHASTIC sweeps to key and resolve each draw
    const uint32_t *ivox, *imask;
};

// Physical parameters in FP64; kernels convert to their compute type.
struct Physics {
    double tau_gas, tau_species;
    double force[3];
    double rho_ref, c_ref;       // storage shifts of the two lattices
    double rho0, c0, c_inlet;
    double p_stick, p;
    double in_scale, in_unscale;  // 2^S and 2^-S of the fixed-point In(k) sums
    int32_t sputter, coupling, species_x, storage;
    double p_stick_product;       // p_S^P
    int32_t product;              // 1: the product lattice P is evolved
    int32_t rounding;             // ROUND_*: how 16-bit stores round (ignored by FP32 and FP64 storage)
    double wall_diffuse;          // sigma: diffuse fraction of the carrier's wall reflection
    uint64_t seed;                // STOCHASTIC: Philox key
    uint32_t step_ctr;            // STOCHASTIC: step whose collision produces the arrivals a launch sums
    uint32_t emission_gather;     // 1: the compact sweep gathers emission reads through LDS where that applies
    double store_ux;              // the carrier is stored and relaxed as h_i - 3 c_ix store_ux (D3Q19; 0 with FP32 storage)
};

// Device buffers of the product lattice for one step (all null / unused when
// the lattice is off).  P populations are stored unshifted (h_i = f_i / w_i),
// 19 direction arrays of nfp elements in the slot order of the pair buffers.
struct ProdStep {
    const void *fin;             // P post-collision populations the sweep pulls from
    void *fout;                  // and the buffer it writes
    void *emit;                  // E_P(k) per interface node (not used by BOUNCEBACK)
    unsigned long long *inacc;   // In_P(k), fixed point like In(k)
    double *acc;                 // sum_t In_P(k, t)
    double *part_sweep;          // 3 per sweep block
    double *pi_now, *pi_prev;    // interface partials (1 per interface block) of steps t and t - 1
};

// Interface list (catalytic nodes with b(k) >= 1), sorted by voxel index.
struct Interface {
    const uint32_t *vox;    // linear voxel index of node k
    const uint32_t *mask;   // bit j (kernel direction numbering): j is an active link
    const double *scale;    // 1/b(k) (UNIFORM) or 1/sum_{active} w_opp(j) (WEIGHTED)
    double *acc;            // sum_t In(k, t)
    // In(k) = sum_j f*_j(k - c_j) of the last sweep, accumulated by that sweep
    // with integer atomics as round(term * 2^S) (two's complement); an
    // integer sum is the same in any order, so results are deterministic.
    unsigned long long *inacc;
    int64_t n;
};

int storage_bytes(int storage);

// Traversal table for the sweep: tiles of `ytile` x-rows in y, z-planes in
// order inside a tile, rows in y, then the chunks of a row.  A row's
// z-neighbours are then ytile rows apart in launch order, inside the set of
// blocks an XCD has in flight, so the populations they share are still in its
// L2.
void build_order(int nx, int ny, int nz, int ytile, uint32_t *order);

// All launchers queue on `stream` and return the launch status.
hipError_t launch_init(const Geometry &g, const Physics &ph, void *pre, void *post, hipStream_t s);
// In(k) of every interface node from a post-collision population buffer (after
// create and after a checkpoint load; during stepping the sweep accumulates it).
hipError_t launch_in_init(const Geometry &g, const Physics &ph, const Interface &it, const void *fin, hipStream_t s);
// In_P(k) from a P post-collision buffer into `inacc` (same terms, unshifted).
hipError_t launch_in_init_product(const Geometry &g, const Physics &ph, const Interface &it, const void *finP,
                                  unsigned long long *inacc, hipStream_t s);
hipError_t launch_sweep(const Geometry &g, const Physics &ph, const void *fin, void *fout, const void *emit,
                        double *part, hipStream_t s);
// The node-compact sweep (same results; needs g.pos and g.worder).
hipError_t launch_sweep_c(const Geometry &g, const Physics &ph, const void *fin, void *fout, const void *emit,
                          double *part, hipStream_t s, const ProdStep *prod = nullptr);
int64_t sweep_blocks_c(const Geometry &g);
// mode 1: moments after streaming fin (fields at step >= 1); mode 2: local
// moments of fin (the initial state, step 0).  Outputs are float arrays, or
// double arrays when out_f64 is set; any output may be null.
hipError_t launch_fields(const Geometry &g, const Physics &ph, const void *fin, const void *emit, int mode,
                         void *rho, void *u, void *conc, bool out_f64, hipStream_t s);
// The same for the x-rows [row0, row1) only, written from index 0 of each
// output with velocity component stride cs.
hipError_t launch_fields_rows(const Geometry &g, const Physics &ph, const void *fin, const void *emit, int mode,
                              void *rho, void *u, void *conc, bool out_f64, int64_t row0, int64_t row1, int64_t cs,
                              hipStream_t s);
// Allocation-free field readback: the device scratch (FIELDS_SCRATCH_DOUBLES
// doubles, one copy per GPU) and the address of `device`'s copy, which must
// be the current device at the first call for it.
constexpr int64_t FIELDS_SCRATCH_DOUBLES = int64_t(4) << 20;  // 32 MiB
constexpr int MAX_SCRATCH_DEVICES = 64;
hipError_t scratch_address(int device, double **out);
// Whether the compact sweep's emission gather is a choice for this storage,
// sputter mode and product setting (FP32 / FP64, UNIFORM / WEIGHTED, no
// product lattice); elsewhere the emission tunable has no effect.
bool emission_gather_applies(int storage, int sputter, bool product);
// Streaming device copy of `bytes` (a multiple of 16, 16-byte aligned).
hipError_t launch_stream_copy(void *dst, const void *src, size_t bytes, hipStream_t s);
// Pull-streaming reference pass (no collision) over a dense periodic lattice
// in the blocked layout, one element of pair_bytes (4, 8 or 16) per direction
// and node; each buffer holds stream_pull_elements(nx, ny, nz) elements.
uint64_t stream_pull_elements(int nx, int ny, int nz);
hipError_t launch_stream_pull(void *dst, const void *src, int nx, int ny, int nz, int pair_bytes, hipStream_t s);
// A box of voxels: origin and extent, inside the lattice.
struct Window {
    int32_t x0, y0, z0, wx, wy, wz;
};
// Pre-collision populations (mode as for launch_fields) of the voxels in
// `win`, FP64, direction-major [19][wz][wy][wx] in the library's numbering.
hipError_t launch_populations(const Geometry &g, const Physics &ph, const void *fin, const void *emit, int mode,
                              const Window &win, double *fC, double *fR, hipStream_t s);
// Product concentration rho_P of every voxel (double, solid 0), from the
// moments after streaming `finP` (mode 1) or of `finP` itself (mode 2); the
// pair buffer `fin` supplies the reactant of reversal re-emission.
hipError_t launch_product_field(const Geometry &g, const Physics &ph, const void *fin, const void *finP,
                                const void *emitP, int mode, double *concP, hipStream_t s);
// phi[x] = sum over the (y, z) plane of concP * u_x (double fields, u
// component-major), one block per x in a fixed order.
hipError_t launch_flux_profile(const Geometry &g, const double *concP, const double *u, double *phi, hipStream_t s);
// Two-stage fixed-order reduction of the per-block partials: FOLD_BLOCKS
// blocks fold contiguous slices into `fold` (FOLD_BLOCKS * NPART doubles),
// then one block sums those and updates the totals.
constexpr int FOLD_BLOCKS = 256;
// One launch for everything of a step but the sweep: the interface kernel of
// step t (iface_blocks blocks, partials to pi_now), when `fold` the first
// reduction stage of step t - 1 (sweep partials ps, interface partials
// pi_prev, into fold_prev), and when `reduce` the final stage of step t - 2
// (from fold_prev2 into tot).  Zero blocks: nothing is launched.
hipError_t launch_front(const Physics &ph, const Interface &it, void *emit, int64_t iface_blocks, double *pi_now,
                        const double *ps, int64_t ns, const double *pi_prev, int64_t ni, double *fold_prev,
                        bool fold, const double *fold_prev2, bool reduce, DevTotals *tot, hipStream_t s,
                        const ProdStep *prod = nullptr);

int64_t sweep_blocks(const Geometry &g);
int64_t interface_blocks(int64_t n);

// One sample of a batch as the host describes it.  block0 / iblock0 are the
// first global logical sweep / interface blocks of the sample; its blocks use
// part_sweep / part_iface exactly as a single-sample step does.
struct BatchSample {
    Geometry g;
    Interface it;
    Physics ph;
    void *pop[2];
    void *emit;
    double *part_sweep, *part_iface;
    uint32_t block0, iblock0;
};

// Per-sample inputs of the batched reduction (the same two stages as in launch_front).
struct ReduceK {
    const double *ps;
    int64_t ns;
    const double *pi;
    int64_t ni;
    double *fold;
    double p, p_stick;
    DevTotals *tot;
};

// Size of one device record of a batch sample, and the upload of n records
// built from `smp` (synchronous on `s`).
size_t batch_record_bytes(int storage);
hipError_t batch_upload(int storage, const BatchSample *smp, int n, void *d_records, hipStream_t s);
// The batched sweep alone (reads buffer `parity` of every sample).  gather:
// the compact sweep gathers its emission reads through LDS where that
// applies (emission_gather_applies).
hipError_t launch_batch_sweep(int storage, int sputter, int species_x, bool compact, bool gather,
                              const void *d_records, const uint32_t *sweep_sample, int64_t sweep_blocks_total,
                              int parity, hipStream_t s);
// One step of every sample: batched interface, sweep (reading population
// buffer `parity` of every sample, writing the other) and reduction.
hipError_t launch_batch_step(int storage, int sputter, int species_x, bool compact, bool gather, const void *d_records,
                             const uint32_t *sweep_sample, int64_t sweep_blocks_total, const uint32_t *iface_sample,
                             int64_t iface_blocks_total, const ReduceK *d_reduce, int n, int parity, hipStream_t s,
                             hipEvent_t sweep_start = nullptr, hipEvent_t sweep_stop = nullptr);

}  // namespace lbmk
