/*
 * lbm.h - C ABI of the MI355X (gfx950) reactive lattice-Boltzmann library.
 *
 * The library advances two D3Q19 lattices over a voxelised porous solid: the
 * carrier gas C and the reactant species R.  One step is the fused pull-
 * streaming + BGK collision of both lattices (Falcucci et al., "Mapping
 * Reactive Flow Patterns in Monolithic Nanoporous Catalysts", Appendix
 * "Numerical Method", Eq. LBE with the second-order equilibrium and the
 * moment equations), halfway bounce-back at solid links, and the paper's
 * "sputtering" stick-and-react boundary condition at every gas-catalyst link
 * (Appendix, eqnarray f_R_in / f_P_in and the text that follows it).
 *
 * Conventions for every entry point:
 *   - Every function returns lbm_status (LBM_OK = 0) except lbm_last_error
 *     and lbm_destroy; nothing throws across the ABI.
 *   - On error the context keeps its previous state and lbm_last_error(ctx)
 *     describes the failure; a failed create sets *out = NULL, leaks nothing
 *     and leaves its message in lbm_last_error(NULL) (thread-local).
 *   - Host pointers are caller-owned; the library copies what it keeps
 *     (voxels, parameter structs) during create.  Device memory is owned by
 *     the context until lbm_destroy.
 *   - A context is not thread-safe.  Work is queued on the context's HIP
 *     stream; calls that return host data synchronise that stream.
 *   - Arrays over voxels are C order (z, y, x) with x (the flow axis) fastest:
 *     node = (z * ny + y) * nx + x.  Vector fields are component-major:
 *     u[a * nnodes + node], a = x, y, z.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = 1,        /* invalid argument (range, NULL, inconsistent) */
    LBM_ENOMEM = 2,        /* host or device allocation failed */
    LBM_EDEVICE = 3,       /* HIP runtime error (no device, launch failure) */
    LBM_ESTATE = 4,        /* call not valid in the context's state */
    LBM_ENONFINITE = 5,    /* a global total became NaN or Inf (state kept) */
    LBM_EUNSUPPORTED = 6   /* valid request this build does not provide */
} lbm_status;

/* Voxel values. */
enum { LBM_FLUID = 0, LBM_INERT = 1, LBM_CATALYTIC = 2 };

/* Sputtering matrix S_ij (probability that reactant arriving along j
 * re-enters along i, with sum_i S_ij = 1; Appendix, text after the
 * sputtering equations).  The paper calls S random.  UNIFORM, WEIGHTED and
 * BOUNCEBACK evolve an expectation: UNIFORM gives each active direction of
 * the node 1/b(k), WEIGHTED gives direction i the share w_i / sum_{active} w,
 * BOUNCEBACK reverses each arrival (S = reversal).  STOCHASTIC draws S: each
 * arrival at node k along active link j leaves whole along one of the b(k)
 * exit directions, each with probability 1/b(k) (expectation: UNIFORM), by
 * Philox4x32-10 (Salmon et al., SC 2011) with key (seed low 32 bits, seed
 * high 32 bits) and counter (step whose collision produced the arrival,
 * voxel index of k, code(j), 0); the first output word r picks exit number
 * floor(r b / 2^32) in ascending code order, code(c) = 9 (c_x + 1) +
 * 3 (c_y + 1) + (c_z + 1).  Runs are reproducible for a given seed; the
 * step enters the counter modulo 2^32.  Not with the product lattice or in
 * batches (LBM_EUNSUPPORTED). */
typedef enum {
    LBM_SPUTTER_UNIFORM = 0, LBM_SPUTTER_WEIGHTED = 1, LBM_SPUTTER_BOUNCEBACK = 2, LBM_SPUTTER_STOCHASTIC = 3
} lbm_sputter;

/* Velocity in the species equilibrium.  PASSIVE: the carrier velocity
 * (j_C + F/2) / rho_C (reactant passively transported by the carrier,
 * "Results & Discussion", initial and inlet conditions).  BARYCENTRIC: the
 * common velocity (j_C + j_R + F/2) / (rho_C + rho_R) of the moment
 * equations, used by both lattices. */
typedef enum { LBM_COUPLE_PASSIVE = 0, LBM_COUPLE_BARYCENTRIC = 1 } lbm_coupling;

/* Species boundary along x.  PERIODIC wraps x like y and z.  RESERVOIR puts
 * an inlet ghost plane at x = -1 holding the rest equilibrium w_i c_inlet
 * (the paper injects reactant at x = 0) and an outlet ghost plane at x = nx
 * that copies plane nx - 1 (zero gradient; where that plane is solid the
 * ghost reflects like inert solid).  INFLOW is RESERVOIR with the inlet ghost
 * moving with the carrier: a node at x = 0 pulls the equilibrium of c_inlet at
 * its own carrier velocity (j_C + F/2) / rho_C, from the carrier populations
 * it has just pulled, so the reservoir injects with the flow; in strongly
 * advective flow RESERVOIR lets less than c_inlet in (0.79 c_inlet at cell
 * Peclet number 5).  The carrier is always periodic. */
typedef enum { LBM_XBC_PERIODIC = 0, LBM_XBC_RESERVOIR = 1, LBM_XBC_INFLOW = 2 } lbm_xbc;

/* Population storage.  All formats store the normalised deviation
 * h_i = f_i / w_i - rho_ref of each population from the rest equilibrium of
 * the reference density (rho_ref = rho0 for the carrier, c_ref for the
 * species).  F32, F16 and BF16 compute in FP32; F64 stores and computes in
 * FP64 (a reference build).  16-bit formats round as lbm_bc.rounding says.
 * The carrier's deviation can also drop a reference flow (lbm_bc.store_ux). */
typedef enum { LBM_STORE_F32 = 0, LBM_STORE_F16 = 1, LBM_STORE_BF16 = 2, LBM_STORE_F64 = 3 } lbm_storage;

/* Rounding of 16-bit stores (F16, BF16; FP32 and FP64 storage ignore it).
 * NEAREST rounds every stored population and emission value to nearest
 * (ties away from zero).  STOCHASTIC rounds each one up with probability
 * equal to the discarded fraction of its last place, so the stored value is
 * right on average: a steady flow no longer sees the same rounding error at
 * the same node every step, which would act on it like a small persistent
 * body force.  The random words are a hash of (step, storage index of the
 * node or interface node, lbm_bc.seed), so runs are reproducible and the
 * In(k) sums still count exactly the stored values.  Not available in batches
 * (LBM_EUNSUPPORTED), whose captured graphs replay the step key. */
typedef enum { LBM_ROUND_NEAREST = 0, LBM_ROUND_STOCHASTIC = 1 } lbm_rounding;

/*
 * Velocity set.  D3Q19 (default) runs every option of this header.  D2Q9 is
 * the paper's own lattice (Appendix "Numerical Method", Fig. A1: weights 4/9,
 * 1/9, 1/36; a catalytic node has at most 8 active links) on one plane:
 * geometry nz = 1, FP64 storage and arithmetic, sputter UNIFORM, WEIGHTED or
 * BOUNCEBACK, either coupling, every species x-boundary, the product
 * lattice, the diffuse or Kn-derived carrier wall.  On a D2Q9 context
 * lbm_step, lbm_fields, lbm_conversion_map, lbm_product_fields, lbm_totals,
 * lbm_query, lbm_active_links, lbm_synchronize and lbm_destroy work as
 * documented (u_z = 0); the other entry points return LBM_EUNSUPPORTED, and
 * batches take D3Q19 samples only.  A non-finite total is reported by
 * lbm_totals (LBM_ENONFINITE).
 */
typedef enum { LBM_LATTICE_D3Q19 = 0, LBM_LATTICE_D2Q9 = 1 } lbm_lattice;

typedef struct {
    int32_t nx, ny, nz;       /* lattice size, each >= 1; nx <= 4096 */
    int32_t reserved0;
    const uint8_t *voxels;    /* host, nx*ny*nz values in {0, 1, 2}; copied */
    double pore_size;         /* delta of Eq. (knudsen) and Eq. (Da_def), > 0 */
} lbm_geometry;

typedef struct {
    int32_t sputter;          /* lbm_sputter */
    int32_t coupling;         /* lbm_coupling */
    int32_t species_x;        /* lbm_xbc */
    int32_t storage;          /* lbm_storage */
    double p_stick;           /* reactant sticking probability p_S^R in [0, 1]
                                 (Table 1 uses 0.95) */
    double c_inlet;           /* reservoir concentration (RESERVOIR, INFLOW), >= 0 */
    double rho0;              /* initial carrier density, > 0 */
    double c0;                /* initial species concentration, >= 0 (the paper
                                 starts with no reactant) */
    double c_ref;             /* species storage shift; < 0 selects 0
                                 (unshifted: best relative precision where
                                 the concentration is depleted) */
    double force[3];          /* body-force density on the carrier (Guo
                                 forcing, half-force velocity shift) */
    int32_t product;          /* 1: also evolve the product lattice P (second
                                 line of the sputtering equations); 0: carrier
                                 and reactant only.  P starts at 0, no product
                                 enters at the inlet, it relaxes with
                                 tau_species and is advected by the carrier.
                                 Needs PASSIVE coupling and the node-compact
                                 sweep (ny, nz <= 1024), LBM_EUNSUPPORTED
                                 otherwise; not available in batches */
    int32_t rounding;         /* lbm_rounding of 16-bit stores (0 = NEAREST) */
    double p_stick_product;   /* product sticking probability p_S^P in [0, 1]
                                 (the paper uses 0); ignored without product */
    uint64_t seed;            /* key of the STOCHASTIC draws and of the
                                 stochastic rounding words; ignored otherwise */
    double wall_diffuse;      /* sigma in [0, 1]: diffuse fraction of the carrier's
                                 reflection at solid walls (Maxwell's
                                 accommodation; lattice Boltzmann form of
                                 Ansumali and Karlin, Phys. Rev. E 66, 026311,
                                 2002).  A gas node's populations pulled from
                                 solid sources keep 1 - sigma of their
                                 bounce-back values and take sigma of the mass
                                 the node sent into the wall, in proportion to
                                 w_i; 0 = halfway bounce-back.  Rarefaction (Kn)
                                 enters through tau_gas.  Not with the product
                                 lattice or in batches (LBM_EUNSUPPORTED) */
    double wall_accommodation;/* sigma_v in [0, 1]; 0: sigma is wall_diffuse.
                                 > 0: sigma is derived from Kn (wall_diffuse
                                 must be 0, LBM_EINVAL otherwise) so that
                                 force-driven flow between two planes
                                 pore_size nodes apart has Maxwell's
                                 first-order slip length ((2 - sigma_v) /
                                 sigma_v) Kn delta (J. C. Maxwell, Phil. Trans.
                                 R. Soc. 170, 231, 1879; Kn of Eq. (knudsen)):
                                 the lattice wall's exact slip length is
                                 sigma (2 tau - 1) / (2 (2 - sigma))
                                 + (16 tau^2 - 16 tau + 1) / (12 delta).
                                 Clamped to [0, 1] where no sigma reaches
                                 Maxwell's slip (bounce-back already slips
                                 more at large tau); lbm_info reports the
                                 value and the clamp.  Same restrictions as
                                 wall_diffuse */
    int32_t lattice;          /* lbm_lattice (0 = D3Q19) */
    int32_t reserved_bc;      /* must be 0 */
    double store_ux;          /* reference flow: x-velocity U, |U| < 0.2
                                 (LBM_EINVAL otherwise).  The carrier is
                                 stored and relaxed in the shifted form
                                 h_i = f_i / w_i - rho_ref - 3 c_ix U: its
                                 deviation from the rest equilibrium minus the
                                 part linear in U (the equilibrium takes the
                                 same shift, the moments add U back).  In a
                                 flow with mean x-velocity near U the values
                                 stored and computed, and with them their
                                 rounding errors, shrink; the results are the
                                 same for any U up to that rounding.  0 =
                                 unshifted.  FP16, BF16 and FP64 storage;
                                 ignored by FP32 storage (whose sweep has no
                                 registers to spare for it) and by the D2Q9
                                 lattice */
} lbm_bc;

/* Optional device hooks.  stream: a hipStream_t all work is queued on
 * (NULL = the null stream).  alloc/free: device allocator used for every
 * device buffer of the context (NULL = hipMalloc/hipFree), e.g. the PyTorch
 * caching allocator.  The struct is copied; user is passed back verbatim. */
typedef struct {
    void *stream;
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, void *user);
    void *user;
} lbm_device;

typedef struct {
    int64_t step;             /* steps taken since create */
    double mass_gas;          /* sum of rho_C over gas nodes at this step */
    double mass_species;      /* sum of rho_R over gas nodes at this step */
    double converted;         /* cumulative p p_S^R sum_t sum_k In(k, t) */
    double lost;              /* cumulative (1 - p) p_S^R sum_t sum_k In(k, t) */
    double influx;            /* cumulative species pulled from the inlet ghost */
    double outflux;           /* cumulative species leaving through x = -1 and
                                 x = nx, net of what the outlet ghost returned */
    int32_t nonfinite;        /* 1 once any total was NaN or Inf */
    int32_t reserved;
    /* product lattice (0 without it) */
    double mass_product;      /* sum of rho_P over gas nodes at this step */
    double lost_product;      /* cumulative p_S^P sum_t sum_k In_P(k, t): product
                                 that stuck at the catalyst */
    double product_out_inlet; /* cumulative product leaving through x = -1 */
    double product_out_outlet;/* cumulative product leaving through x = nx, net
                                 of what the outlet ghost returned; over a
                                 window, its increase over that of influx is
                                 the conversion efficiency of Eq. (eff) */
} lbm_totals_t;

typedef struct {
    double tau_gas, tau_species;   /* relaxation times in use */
    double kn;                     /* Kn = cs (tau_gas - 1/2) / delta */
    double p;                      /* reaction probability in use */
    double da;                     /* Damkohler number requested */
    double pore_size;
    int32_t p_clamped;             /* 1 when cs / (Da delta) exceeded 1 */
    int32_t storage;
    int64_t n_nodes;               /* nx * ny * nz */
    int64_t n_fluid;               /* gas nodes */
    int64_t n_interface;           /* catalytic nodes with b(k) >= 1 */
    int64_t n_catalytic_links;     /* sum_k b(k) */
    int64_t device_bytes;          /* device memory held by the context */
    double wall_sigma;             /* diffuse fraction of the gas wall in use */
    int32_t wall_clamped;          /* 1 when the Kn relation clamped it to [0, 1] */
    int32_t reserved_info;
} lbm_info;

/* Per-kernel device time accumulated while timing is enabled.
 * sweep: the fused stream-collide sweep, once per step.
 * interface: the launch before each sweep, which runs the interface kernel of
 *   the step together with the first reduction stage of the previous step and
 *   the final stage of the one before (when those belong to the same
 *   lbm_step call).
 * reduce: the reductions that close an lbm_step call (after its last sweep);
 *   n_reduce counts calls.
 * xflux: unused (the sweep tallies the reservoir planes), always 0. */
typedef struct {
    double ms_sweep, ms_interface, ms_xflux, ms_reduce;
    int64_t n_sweep, n_interface, n_xflux, n_reduce;
} lbm_kernel_times_t;

/*
 * lbm_create / lbm_create_on - build a simulation context.
 *
 * g:    geometry; voxels 0 gas, 1 inert solid, 2 catalytic solid.  Per the
 *       paper every solid node in contact with gas acts catalytically when
 *       flagged 2 (Appendix, text after the sputtering equations); a
 *       catalytic node k receives along its active links j, those whose pull
 *       source k - c_j is a gas node inside the domain; b(k) counts them.
 * kn:   Knudsen number, Eq. (knudsen): Kn = cs (tau - 1/2) / delta.  Used to
 *       derive tau_gas = 1/2 + Kn delta / cs when tau[0] == 0.  kn == 0 means
 *       "not given"; when both are given they must agree to 1e-9 relative.
 * da:   Damkohler number, Eq. (Da_def), with tau_ch = 1/p and
 *       tau_tr = delta / cs ("Results & Discussion"): p = cs / (Da delta),
 *       clamped to 1 (p_clamped set); da = +inf gives p = 0.  da must be > 0.
 * tau:  {tau_gas, tau_species}; 0 = derive (tau_gas from kn, tau_species =
 *       tau_gas: the paper takes tau equal for all species); otherwise > 1/2.
 * bc:   boundary and storage options, see lbm_bc.
 * dev:  (lbm_create_on) device hooks, may be NULL.
 * out:  receives the context.
 *
 * Errors: LBM_EINVAL for NULL pointers, sizes < 1, nx > 4096, a voxel > 2,
 * tau <= 1/2, kn < 0, da <= 0 or NaN, inconsistent kn/tau, p_stick outside
 * [0, 1], c_inlet/c0 < 0, rho0 <= 0, an unknown rounding, nonzero reserved
 * fields;
 * LBM_EUNSUPPORTED for an unknown enum value, or for a lattice whose
 * buffers exceed the kernels' 32-bit offsets (4 * nfp * s >= 2^32 bytes with
 * nfp = gas nodes + 1 rounded up to 128 and s the bytes per stored
 * population, an emission array of 2^32 bytes or more, or 2^30 gas or
 * interface nodes); LBM_EDEVICE without a usable gfx950 device; LBM_ENOMEM
 * when a buffer cannot be allocated.
 */
lbm_status lbm_create(const lbm_geometry *g, double kn, double da, const double tau[2],
                      const lbm_bc *bc, lbm_ctx **out);
lbm_status lbm_create_on(const lbm_geometry *g, double kn, double da, const double tau[2],
                         const lbm_bc *bc, const lbm_device *dev, lbm_ctx **out);

/*
 * lbm_inspect - what lbm_create would build, without a device: the same
 * argument checks (same errors) and parameter maps (tau, Kn, p, p_clamped),
 * the node, interface-node and catalytic-link counts, and the device bytes the
 * context would allocate (populations, emission, tables, partial sums; within
 * 256 B per buffer).  Host memory only; usable on a machine without a GPU.
 */
lbm_status lbm_inspect(const lbm_geometry *g, double kn, double da, const double tau[2],
                       const lbm_bc *bc, lbm_info *info);

/*
 * lbm_step - advance n >= 0 time steps (Eq. LBE for both lattices plus the
 * sputtering boundary condition).  Asynchronous on the context stream.
 * Returns LBM_ENONFINITE if a total of an earlier, completed step was found
 * non-finite (detection lags by at most one call; lbm_totals reports it
 * exactly); LBM_EINVAL for n < 0.
 */
lbm_status lbm_step(lbm_ctx *c, int64_t n);

/*
 * lbm_fields - moments of the pre-collision populations at the current step
 * (moment equations of the Appendix): rho = rho_C, u = the velocity of the
 * coupling mode (PASSIVE: (j_C + F/2) / rho_C), conc = rho_R.  Host arrays of
 * n_nodes doubles (u: 3 * n_nodes, component-major); any may be NULL.  Solid
 * voxels read 0.  Synchronises the stream.
 */
lbm_status lbm_fields(lbm_ctx *c, double *rho, double *u, double *conc);

/* Same moments written to device arrays of float (n_nodes, 3 * n_nodes,
 * n_nodes), queued on the context stream without synchronising. */
lbm_status lbm_fields_device(lbm_ctx *c, float *rho, float *u, float *conc);

/* lbm_fields_noalloc - lbm_fields for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same outputs, bit for bit, through a fixed device
 * scratch instead of temporary buffers.  Calls no hipMalloc or hipFree and
 * takes nothing from lbm_device.alloc.
 *
 * rho, u (3 N, component-major), conc: host, caller-owned, N = nx ny nz
 * doubles each (u: 3 N); NULL = skip.  Synchronises the context's stream.
 * The fields pass through a 32 MiB device array (one per GPU, held until the
 * process ends) in passes of whole x-rows, 5 nx doubles a row.  Calls on one
 * GPU share that array: calls that overlap in time on one GPU (from several
 * threads or streams) race and must be serialised by the caller.  Makes the
 * context's device current for the call and restores the caller's.
 * Errors: LBM_EINVAL for a NULL context or an x-row that does not fit the
 * scratch (not reachable with nx <= 4096); LBM_EDEVICE when the scratch
 * cannot be resolved on the device or a launch or copy fails. */
lbm_status lbm_fields_noalloc(lbm_ctx *c, double *rho, double *u, double *conc);

/* lbm_stream_copy - the HBM streaming reference that the sweep's bandwidth
 * is reported against (not part of the method): copies `bytes` from src to
 * dst, both device memory, on `stream` (NULL = the null stream),
 * asynchronously, one 16-byte element per thread with non-temporal loads and
 * stores.  bytes and both pointers must be multiples of 16 (LBM_EINVAL);
 * the buffers must not overlap.  LBM_EDEVICE when the launch fails. */
lbm_status lbm_stream_copy(void *dst, const void *src, size_t bytes, void *stream);

/* lbm_stream_pull - the streaming reference for the sweep's own access
 * pattern (not part of the method): one pull-streaming pass of D3Q19 with no
 * collision over a dense periodic nx x ny x nz lattice, in the blocked
 * population layout the sweep uses.  Node n = x + nx (y + ny z) of the
 * lattice reads element i of its upwind neighbour (x - c_ix, y - c_iy,
 * z - c_iz), periodic in all three axes, and writes it to its own slot i:
 * the population traffic of a sweep over a lattice of gas nodes only, one
 * pair of pair_bytes per direction and node.
 * Layout of src and dst (device memory, caller-owned, each
 * ceil(nx ny nz / 64) * 64 * 19 * pair_bytes bytes): element (n, i) at
 * index (n / 64) * 1216 + 64 i + n % 64.  pair_bytes: 4 (16-bit storage),
 * 8 (FP32) or 16 (FP64).  Asynchronous on `stream` (NULL = the null stream).
 * Errors: LBM_EINVAL for NULL or misaligned pointers, overlapping buffers,
 * sizes below 1, ny or nz above 65535, more than 2^27 nodes, or another
 * pair_bytes; LBM_EDEVICE when the launch fails. */
lbm_status lbm_stream_pull(void *dst, const void *src, int32_t nx, int32_t ny, int32_t nz, int32_t pair_bytes,
                           void *stream);

/*
 * lbm_conversion_map - per voxel, the reactant converted at that catalytic
 * node so far: p p_S^R sum_t In(k, t), where In(k, t) is everything arriving
 * at k along its active links in step t (second line of the sputtering
 * equations: the source of product).  0 at gas and inert voxels.  Host array
 * of n_nodes doubles.  Synchronises the stream.
 */
lbm_status lbm_conversion_map(lbm_ctx *c, double *conv);

/*
 * lbm_product_fields - product-lattice outputs at the current step (contexts
 * created with bc.product = 1; LBM_EUNSUPPORTED otherwise).  Host arrays, any
 * may be NULL:
 *   conc  n_nodes doubles, rho_P of the pre-collision populations ([z][y][x],
 *         solid 0);
 *   stuck n_nodes doubles, p_S^P sum_t In_P(k, t): product that stuck at
 *         catalytic node k (0 elsewhere);
 *   phi   nx doubles, the product flux profile Phi_P along the flow
 *         ("Results & Discussion"): phi[x] = sum over the (y, z)
 *         cross-section of rho_P u_x, u the carrier velocity (j_C + F/2) /
 *         rho_C.
 * Synchronises the stream; allocates temporary device memory for phi.
 */
lbm_status lbm_product_fields(lbm_ctx *c, double *conc, double *stuck, double *phi);

/*
 * lbm_populations - the pre-collision populations f_i of both lattices at the
 * current step (the state Eq. LBE advances) in a box of voxels: origin
 * {x0, y0, z0}, extent {wx, wy, wz} >= 1, inside the lattice (LBM_EINVAL
 * otherwise).  fC and fR are host arrays of 19 * wx * wy * wz doubles,
 * direction-major: f[i][z][y][x] relative to the origin; solid voxels are 0.
 * Direction numbering: i = 0 rest; i = 1..9 are (1,0,0), (0,1,0), (0,0,1),
 * (1,1,0), (1,-1,0), (1,0,1), (1,0,-1), (0,1,1), (0,1,-1); i = 10..18 are the
 * negatives of i - 9.  Synchronises the stream.
 */
lbm_status lbm_populations(lbm_ctx *c, const int32_t origin[3], const int32_t extent[3], double *fC,
                           double *fR);

/* Global totals (FP64, fixed-order deterministic reductions). Synchronises. */
lbm_status lbm_totals(lbm_ctx *c, lbm_totals_t *t);

/* Parameters in use and sizes. */
lbm_status lbm_query(const lbm_ctx *c, lbm_info *info);

/* b(k) per voxel (0 for non-catalytic voxels), host array of n_nodes bytes. */
lbm_status lbm_active_links(const lbm_ctx *c, uint8_t *b);

/* Wait for all work queued by the context. */
lbm_status lbm_synchronize(lbm_ctx *c);

/* Launch-shape tunables.
 * LBM_TUNE_YTILE: rows per y-tile of the sweep traversal, 1..ny (default
 * 16).  The sweep walks tiles of that many x-rows in y, z-planes inside a
 * tile, so a row's z-neighbours are read while still cached.  Results do not
 * depend on it.
 * LBM_TUNE_SWEEP: 1 (default where available) = node-compact sweep, one lane
 * per gas node; 0 = one wavefront per 64-voxel chunk of an x-row (solid
 * voxels leave lanes idle).  The two compute the same values; the totals
 * may differ in the last bits (per-block partial sums group nodes
 * differently).  The compact sweep needs ny, nz <= 1024 (LBM_EUNSUPPORTED
 * otherwise).
 * LBM_TUNE_EMISSION: how the compact sweep reads the emission values of its
 * catalytic sources: 1 (default for a context) = each full wavefront lists
 * its sources in LDS and reads them 64 per pass; 0 = one read per direction
 * and lane.  Both read the same values, so every result is bit-identical.
 * It has an effect only with FP32 or FP64 storage, UNIFORM or WEIGHTED
 * sputtering and no product lattice; elsewhere the value is kept and
 * ignored. */
typedef enum { LBM_TUNE_YTILE = 0, LBM_TUNE_SWEEP = 1, LBM_TUNE_EMISSION = 2 } lbm_tunable;
lbm_status lbm_set_tunable(lbm_ctx *c, int32_t which, int64_t value);   /* LBM_EINVAL: unknown or out of range */
lbm_status lbm_get_tunable(const lbm_ctx *c, int32_t which, int64_t *value);

/*
 * lbm_autotune - pick the launch shape: time `reps` (1..1000) sweeps for each
 * candidate (sweep variant x y-tile in {4, 8, 16, 32, 64, 128}, clamped to
 * ny; for the compact sweep also both LBM_TUNE_EMISSION modes where that
 * tunable has an effect) in two interleaved rounds and keep the candidate
 * with the fastest round.  The trial sweeps run in place; the population
 * buffer and In(k) accumulators they overwrite are saved to temporary device memory
 * first and restored afterwards, so the state (and every later result) is
 * exactly as before the call.  best_ms (may be NULL) receives the mean sweep
 * time of the winner.  Synchronises the stream.
 */
lbm_status lbm_autotune(lbm_ctx *c, int32_t reps, double *best_ms);

/* Per-kernel HIP-event timing on the context's stream: 1 times every launch
 * (eight events per step), 2 the sweep only (two events per step; the other
 * fields stay 0), 0 disables; other values are LBM_EINVAL.  Events between
 * launches cost step time (about 30 us per step with 1 at 256^3 on MI355X),
 * so 2 is the level to use around a throughput measurement.  Reading
 * synchronises the stream.  Reset on enable. */
lbm_status lbm_set_timing(lbm_ctx *c, int32_t enable);
lbm_status lbm_kernel_times(lbm_ctx *c, lbm_kernel_times_t *t);

/*
 * Checkpoint of the full state (populations of every lattice, emission and
 * accumulator arrays, totals, step) with a header that records the geometry
 * hash and the parameters (product lattice and STOCHASTIC seed included);
 * lbm_load requires a context created with the same geometry and parameters
 * (LBM_EINVAL otherwise) and makes the next steps bit-identical to an
 * uninterrupted run.  Synchronise the stream.
 */
lbm_status lbm_save(lbm_ctx *c, const char *path);
lbm_status lbm_load(lbm_ctx *c, const char *path);

/* Message of the last failure on c (c == NULL: the calling thread's last
 * create failure).  Valid until the next call on the same context/thread. */
const char *lbm_last_error(const lbm_ctx *c);

/* Release the context and its device memory.  NULL is a no-op. */
void lbm_destroy(lbm_ctx *c);

/*
 * Batches: many independent samples (each a full context: its own geometry,
 * Kn, Da, tau and boundary options) advanced together, one launch per kernel
 * per step for the whole batch instead of one per sample.  Every sample
 * evolves exactly as it would alone (same kernels and summation order), so
 * its fields, conversion map and totals are bit-identical to a single
 * context created with the same arguments and stepped as often.
 *
 * lbm_batch_create - n >= 1 samples; sample i takes g[i], kn[i] (kn may be
 *       NULL: all "not given"), da[i], tau[i] and bc[i] with the meaning of
 *       lbm_create.  bc[i].storage, .sputter, .coupling and .species_x must
 *       be equal for all samples (LBM_EINVAL otherwise); the other fields,
 *       store_ux included, may differ.  dev as in
 *       lbm_create_on; every sample and the batch use its stream.  A failed
 *       create releases everything, sets *out = NULL and leaves a message
 *       naming the sample in lbm_batch_last_error(NULL).
 * lbm_batch_step - advance every sample n >= 0 steps (asynchronous).  With
 *       graphs enabled (lbm_batch_set_graph) the steps replay captured HIP
 *       graphs: a 64-step loop while at least 64 steps remain, then a 2-step
 *       loop, and an odd last step launched directly.  LBM_ENONFINITE as for
 *       lbm_step, with the sample named in the message.
 * lbm_batch_fields / _conversion_map / _totals / _query - lbm_fields,
 *       lbm_conversion_map, lbm_totals and lbm_query of sample i
 *       (0 <= i < n, LBM_EINVAL otherwise).
 * lbm_batch_set_graph - 1: capture the step in a HIP graph on first use and
 *       replay it; 0 (default): launch directly.  Results are identical.
 */
typedef struct lbm_batch lbm_batch;
lbm_status lbm_batch_create(int32_t n, const lbm_geometry *g, const double *kn, const double *da,
                            const double (*tau)[2], const lbm_bc *bc, const lbm_device *dev,
                            lbm_batch **out);
lbm_status lbm_batch_step(lbm_batch *b, int64_t n);
lbm_status lbm_batch_fields(lbm_batch *b, int32_t i, double *rho, double *u, double *conc);
lbm_status lbm_batch_conversion_map(lbm_batch *b, int32_t i, double *conv);
lbm_status lbm_batch_totals(lbm_batch *b, int32_t i, lbm_totals_t *t);
lbm_status lbm_batch_query(const lbm_batch *b, int32_t i, lbm_info *info);
lbm_status lbm_batch_synchronize(lbm_batch *b);
lbm_status lbm_batch_set_graph(lbm_batch *b, int32_t enable);
/* Tunables of every sample (see lbm_set_tunable).  LBM_TUNE_SWEEP applies to
 * the whole batch (1 needs every sample to support the compact sweep);
 * LBM_TUNE_YTILE is clamped to each sample's ny; get reports sample 0's.
 * LBM_TUNE_EMISSION applies to the batched sweep (default 0 for a batch:
 * direct reads); changing it discards the captured step graphs. */
lbm_status lbm_batch_set_tunable(lbm_batch *b, int32_t which, int64_t value);
lbm_status lbm_batch_get_tunable(const lbm_batch *b, int32_t which, int64_t *value);
/* lbm_autotune for the batched sweep: one variant and y-tile for the batch. */
lbm_status lbm_batch_autotune(lbm_batch *b, int32_t reps, double *best_ms);
/* Sweep timing of a batch, for measurement: lbm_batch_set_timing(b, 2)
 * records HIP events on the batch stream around the batched sweep of every
 * step (0 stops; 1 is not supported, LBM_EINVAL) and resets the sums.
 * While it is on, lbm_batch_step launches every step directly (captured
 * graphs cannot hold the events).  lbm_batch_kernel_times synchronises the
 * stream and reports ms_sweep / n_sweep of the steps since the reset (the
 * other fields zero). */
lbm_status lbm_batch_set_timing(lbm_batch *b, int32_t enable);
lbm_status lbm_batch_kernel_times(lbm_batch *b, lbm_kernel_times_t *t);
const char *lbm_batch_last_error(const lbm_batch *b);
void lbm_batch_destroy(lbm_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
