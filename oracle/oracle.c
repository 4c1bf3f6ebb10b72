/*
 * FP64 reference ("oracle") for the reactive two-lattice lattice-Boltzmann step.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline timing of the benchmark load this library.  The product path (the
 * HIP library and its Python binding) never links, imports or calls it, and it
 * shares no code, header or table with that path.
 *
 * Plain, slow and obviously correct on purpose: array-of-structures storage
 * f[node][Q], one loop per step of the method, FP64 throughout, a fixed
 * summation order (directions ascending, nodes in (z, y, x) order, interface
 * nodes in index order).  The only parallelism is OpenMP over z-planes in the
 * collision and streaming loops, where every node writes only its own entries,
 * so results are bit-identical for any thread count.
 *
 * What is computed (paper: Appendix "Numerical Method"):
 *   - BGK lattice Boltzmann equation for each species alpha, Eq. (LBE):
 *       f_i(x + c_i, t + 1) - f_i(x, t) = omega [f_i^eq(x, t) - f_i(x, t)],
 *     split as collision followed by streaming;
 *   - second-order equilibrium w_i rho [1 + c.u/cs^2 + (c.u)^2/(2 cs^4)
 *     - u^2/(2 cs^2)] with cs^2 = 1/3 (equilibrium equation after Eq. LBE);
 *   - moments rho = sum_i f_i, rho u = sum_i c_i f_i, and the common
 *     barycentric velocity sum_a rho_a u_a / sum_a rho_a (moment equations);
 *   - the lattice is D3Q19 (weights 1/3, 1/18, 1/36), the 3-D counterpart of
 *     the paper's D2Q9; it meets the paper's weight constraints
 *     sum w = 1, sum w c = 0, sum w c c = cs^2 I.  The same source built with
 *     ORC_D2Q9 defined is the paper's own D2Q9 (weights 4/9, 1/9, 1/36) on
 *     one z-plane: every step below is written for any velocity set, and a
 *     catalytic node then has at most 8 active links;
 *   - the "sputtering" stick-and-react boundary condition, first line of the
 *     eqnarray (f_R_in / f_P_in): a reactant population arriving at a catalytic
 *     node along an active link is re-emitted into the gas with probability
 *     (1 - p_S^R) along the directions picked by the sputtering matrix S,
 *     which conserves what it redistributes (sum_i S_ij = 1); the fraction
 *     p p_S^R is converted into product (second line), the remaining
 *     (1 - p) p_S^R is lost, so total (R + P) mass is not conserved unless the
 *     sticking probability is zero (text after the eqnarray);
 *   - a body force drives the carrier ("Validation of Numerical Model"),
 *     implemented with Guo's forcing term and the half-force velocity shift;
 *   - optionally the product lattice P (second line of the eqnarray): a
 *     catalytic node re-emits into the gas, along the directions picked by
 *     S, the converted reactant p p_S^R In_R(k) plus the fraction
 *     (1 - p_S^P) of the product that arrived there, In_P(k); the fraction
 *     p_S^P of arriving product sticks and leaves the system;
 *   - the diagnostics of "Results & Discussion": the conversion efficiency
 *     (Eq. eff), product mass leaving through the outlet over reactant mass
 *     entering through the inlet, and the product flux profile Phi_P
 *     (Eq. for Phi_P), sum over a cross-section of rho_P u along the flow.
 *
 * Readings where the paper is silent (the same readings the HIP path uses):
 *   - gas lattice C, reactant lattice R and, when enabled, product lattice P;
 *     one relaxation time for the gas and one shared by the two species (the
 *     paper takes tau equal for all species); P starts at zero and the
 *     inlet ghost holds no product (only carrier and reactant are injected);
 *   - species advection velocity: PASSIVE (carrier velocity; the text says
 *     reactant and product are passively transported by the carrier) or
 *     BARYCENTRIC (the common velocity of the moment equations);
 *   - halfway bounce-back at every solid link of the gas, and at inert-solid
 *     links of the species; optionally the gas wall reflects a fraction
 *     sigma diffusely (Maxwell's accommodation model; in lattice Boltzmann
 *     form, Ansumali and Karlin, Phys. Rev. E 66, 026311 (2002)): at a gas
 *     node, the populations pulled from solid sources share the mass the node
 *     sends into the wall, M, in proportion to w_i (the equilibrium of a wall
 *     at rest), f_i = (1 - sigma) f*_opp(i) + sigma w_i M / W, with W the sum
 *     of w_i over those directions; sigma = 0 is bounce-back.  The rarefaction
 *     (Kn) enters through tau; sigma is the wall's accommodation;
 *   - sputter timing: what arrives at a catalytic node during a step leaves it
 *     along the reversed active links at the next streaming (link-wise,
 *     one step, like halfway bounce-back);
 *   - S as an expectation: UNIFORM (each active direction 1/b), WEIGHTED
 *     (proportional to w_i) or BOUNCEBACK (reversal); or S drawn at random
 *     (STOCHASTIC, the paper's random discrete orientation): each arrival at
 *     catalytic node k along active link j leaves whole along one of the b(k)
 *     exit directions {opp(j') : j' active}, picked with probability 1/b(k)
 *     (so the expectation is UNIFORM).  The draw is a pure function of
 *     (seed, step, k, j): Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
 *     "Parallel random numbers: as easy as 1, 2, 3", SC 2011) with key
 *     (seed low, seed high) and counter (step, k, code(j), 0), where code(c)
 *     = 9 (c_x + 1) + 3 (c_y + 1) + (c_z + 1) labels a velocity independently
 *     of any direction numbering; the first output word r picks the exit
 *     floor(r b / 2^32) in ascending code order.  The step is the one whose
 *     collision produced the arriving populations;
 *   - species x-boundaries: RESERVOIR puts an inlet ghost plane at x = -1
 *     holding w_i c_in and an outlet ghost plane at x = nx that copies plane
 *     nx - 1 (zero gradient; a solid copy reflects as inert solid);
 *     INFLOW is the same except that the inlet ghost holds the equilibrium
 *     of c_in moving with the carrier: f_i^eq(c_in, u) with
 *     u = (sum_i c_i f_i^C + F/2) / sum_i f_i^C of the node it feeds, from
 *     the carrier populations that node has just pulled (reactant injected
 *     with the flow, as at the paper's inlet);
 *     PERIODIC wraps x like y and z.  The gas is periodic in x, y and z;
 *   - BARYCENTRIC sums the moments of every lattice present (C, R and P).
 */

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifdef ORC_D2Q9
/* D2Q9, the paper's lattice (Appendix "Numerical Method", Fig. A1): rest
 * (w = 4/9), 4 axis links (w = 1/9), 4 diagonals (w = 1/36), all with c_z = 0;
 * the lattice is one z-plane (nz = 1). */
#define Q 9
static const int CX[Q] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
static const int CY[Q] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
static const int CZ[Q] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
static const double WT[Q] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7};
#else
#define Q 19

/* D3Q19: rest, 6 axis links (w = 1/18), 12 face diagonals (w = 1/36). */
static const int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
static const double WT[Q] = {1.0 / 3.0,
                             1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
#endif

enum { ORC_FLUID = 0, ORC_INERT = 1, ORC_CATALYTIC = 2 };
enum { ORC_UNIFORM = 0, ORC_WEIGHTED = 1, ORC_BOUNCEBACK = 2, ORC_STOCHASTIC = 3 };
enum { ORC_PASSIVE = 0, ORC_BARYCENTRIC = 1 };
enum { ORC_XPERIODIC = 0, ORC_XRESERVOIR = 1, ORC_XINFLOW = 2 };

typedef struct {
    double tau_gas, tau_species; /* relaxation times of C and R */
    double p;                    /* reaction probability */
    double p_stick;              /* sticking probability p_S^R */
    double c_inlet;              /* reservoir concentration */
    double rho0, c0;             /* initial carrier density and concentration */
    double force[3];             /* body-force density on the carrier */
    int32_t sputter, coupling, species_x, pad;
    double p_stick_product;      /* sticking probability p_S^P of the product */
    int32_t product, pad2;       /* 1: evolve the product lattice P */
    uint64_t seed;               /* key of the STOCHASTIC sputter draws */
    double wall_diffuse;         /* sigma: diffuse fraction of the gas wall reflection */
} orc_params;

typedef struct {
    int nx, ny, nz;
    long n;
    unsigned char *vox;
    orc_params prm;
    double *fC, *fR;   /* pre-collision populations f[node*Q + i] */
    double *pC, *pR;   /* post-collision populations */
    double *em;        /* emission E_i(k) of catalytic nodes, [node*Q + i] */
    double *acc;       /* accumulated arrivals sum_t In(k, t), per node */
    double tot[6];     /* mass_gas, mass_species, converted, lost, influx, outflux */
    /* product lattice (NULL unless prm.product) */
    double *fP, *pP, *emP, *accP;
    /* mass_product, lost_product (p_S^P sum In_P), product leaving through
     * the inlet face, product leaving through the outlet face (net) */
    double totp[4];
    long step;
} orc;

/* ---------------------------------------------------------------- tables -- */

/* The velocity set of this build (D3Q19, or D2Q9 when built with
 * ORC_D2Q9): c[3 i + a], w[i], opp[i]; returns Q. */
int orc_d3q19(int *c, double *w, int *opp)
{
    for (int i = 0; i < Q; ++i) {
        c[3 * i + 0] = CX[i];
        c[3 * i + 1] = CY[i];
        c[3 * i + 2] = CZ[i];
        w[i] = WT[i];
        opp[i] = OPP[i];
    }
    return Q;
}

/* ------------------------------------------------------- parameter maps -- */

/* Knudsen number Kn = cs (tau - dt/2) / delta, Eq. (knudsen) with dt = 1. */
double orc_kn_from_tau(double tau, double delta)
{
    return sqrt(1.0 / 3.0) * (tau - 0.5) / delta;
}

double orc_tau_from_kn(double kn, double delta)
{
    return 0.5 + kn * delta / sqrt(1.0 / 3.0);
}

/* Diffuse fraction sigma of the gas wall that gives Maxwell's first-order
 * slip at Knudsen number kn (test infrastructure: the relation the library
 * applies when a tangential accommodation coefficient is given).
 *
 * Maxwell's slip law (J. C. Maxwell, Phil. Trans. R. Soc. 170, 231, 1879):
 * u_s = ((2 - sigma_v) / sigma_v) lambda du/dn at the wall, sigma_v the
 * tangential momentum accommodation coefficient, lambda = Kn delta the mean
 * free path of Eq. (knudsen).  The lattice wall (a fraction sigma reflected
 * diffusely, 1 - sigma bounced back) has its own slip, fixed by tau and
 * sigma; it is found from the exact steady solution of force-driven flow F in
 * a plane channel of N = delta gas nodes with that wall (populations depend
 * on the wall-normal coordinate only; BGK with Guo forcing, halfway walls):
 *   rho u(y) = M0 - (K / 2) (y - y_c)^2,  K = F / nu,  nu = (tau - 1/2) / 3,
 *   M0 = K [ (N - 1)^2 / 8 + N (1 + sigma (tau - 1)) / (2 (2 - sigma))
 *            + (8 tau^2 - 8 tau - 1) / 12 ],
 * y_c the channel centre and the walls halfway outside the first and last
 * gas nodes.  Its value at the wall over the wall shear rate K N / 2 (per rho)
 * is the lattice slip length
 *   l_s = sigma (2 tau - 1) / (2 (2 - sigma)) + (16 tau^2 - 16 tau + 1) / (12 N),
 * and setting l_s = ((2 - sigma_v) / sigma_v) Kn N gives s = sigma / (2 - sigma)
 * in closed form; sigma = 2 s / (1 + s), clamped to [0, 1] (*clamped = 1 when
 * the lattice wall cannot reach Maxwell's slip: below sigma = 0 the
 * bounce-back slip of large tau already exceeds it).  tau follows from kn by
 * Eq. (knudsen). */
double orc_wall_sigma_from_kn(double kn, double delta, double accommodation, int *clamped)
{
    const double tau = orc_tau_from_kn(kn, delta);
    const double N = delta;
    const double A = (2.0 - accommodation) / accommodation;
    const double target = A * kn * N;                                    /* Maxwell slip length */
    const double bb = (16.0 * tau * tau - 16.0 * tau + 1.0) / (12.0 * N); /* slip length of bounce-back */
    const double s = (target - bb) * 2.0 / (2.0 * tau - 1.0);            /* sigma / (2 - sigma) */
    double sigma = 2.0 * s / (1.0 + s);
    int cl = 0;
    if (!(s >= 0.0)) {
        sigma = 0.0;
        cl = 1;
    } else if (sigma > 1.0) {
        sigma = 1.0;
        cl = 1;
    }
    if (clamped) *clamped = cl;
    return sigma;
}

/* Damkohler number Da = tau_ch / tau_tr, Eq. (Da_def), with the chemical time
 * tau_ch = dt / p = 1 / p in lattice units and the transport time
 * tau_tr = delta / v, v taken as the lattice sound speed ("Results &
 * Discussion", definition of the conversion efficiency study).  Hence
 * p = cs / (Da delta), clamped to a probability; Da = +inf gives p = 0. */
double orc_p_from_da(double da, double delta, int *clamped)
{
    double p;
    if (isinf(da))
        p = 0.0;
    else
        p = sqrt(1.0 / 3.0) / (da * delta);
    if (clamped)
        *clamped = p > 1.0;
    return p > 1.0 ? 1.0 : p;
}

double orc_da_from_p(double p, double delta)
{
    return (1.0 / p) / (delta / sqrt(1.0 / 3.0));
}

/* -------------------------------------------------- kinetic ingredients -- */

/* Second-order equilibrium (equilibrium equation of the Appendix), cs^2 = 1/3. */
void orc_equilibrium(double rho, const double *u, double *feq)
{
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        double cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
        feq[i] = WT[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

/* Guo forcing term (1 - 1/(2 tau)) w_i [3 (c_i - u) + 9 (c_i . u) c_i] . F. */
void orc_guo_source(double tau, const double *u, const double *F, double *S)
{
    for (int i = 0; i < Q; ++i) {
        double c[3] = {CX[i], CY[i], CZ[i]};
        double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
        double s = 0.0;
        for (int a = 0; a < 3; ++a)
            s += (3.0 * (c[a] - u[a]) + 9.0 * cu * c[a]) * F[a];
        S[i] = (1.0 - 1.0 / (2.0 * tau)) * WT[i] * s;
    }
}

/* Neumaier-compensated running sum, so that the global totals carry no
 * summation error worth speaking of (a plain serial sum over ~1e6 terms drifts
 * by ~1e-12 relative, which would hide the conservation properties). */
typedef struct {
    double s, c;
} ksum;

static void kadd(ksum *k, double v)
{
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v))
        k->c += (k->s - t) + v;
    else
        k->c += (v - t) + k->s;
    k->s = t;
}

static double kval(const ksum *k)
{
    return k->s + k->c;
}

/* ------------------------------------------------------------- geometry -- */

static long node(const orc *o, int x, int y, int z)
{
    return ((long)z * o->ny + y) * o->nx + x;
}

static int wrap(int a, int n)
{
    a %= n;
    return a < 0 ? a + n : a;
}

/* Source of the pull along direction i into (x, y, z): (x, y, z) - c_i with y
 * and z periodic; x periodic when xper, else returned as is (may be -1 or nx). */
static void source(const orc *o, int x, int y, int z, int i, int xper, int *sx, int *sy, int *sz)
{
    *sx = xper ? wrap(x - CX[i], o->nx) : x - CX[i];
    *sy = wrap(y - CY[i], o->ny);
    *sz = wrap(z - CZ[i], o->nz);
}

/* Incoming active links of catalytic node k: j >= 1 whose source k - c_j is an
 * in-domain gas node.  Returns b(k) and the link set as a bit mask. */
static int active_links(const orc *o, int x, int y, int z, unsigned *mask)
{
    int xper = o->prm.species_x == ORC_XPERIODIC;
    int b = 0;
    *mask = 0;
    for (int j = 1; j < Q; ++j) {
        int sx, sy, sz;
        source(o, x, y, z, j, xper, &sx, &sy, &sz);
        if (sx < 0 || sx >= o->nx)
            continue;
        if (o->vox[node(o, sx, sy, sz)] == ORC_FLUID) {
            *mask |= 1u << j;
            ++b;
        }
    }
    return b;
}

void orc_link_counts(const orc *o, unsigned char *b)
{
    for (int z = 0; z < o->nz; ++z)
        for (int y = 0; y < o->ny; ++y)
            for (int x = 0; x < o->nx; ++x) {
                long n = node(o, x, y, z);
                unsigned m;
                b[n] = o->vox[n] == ORC_CATALYTIC ? (unsigned char)active_links(o, x, y, z, &m) : 0;
            }
}

/* ------------------------------------------------------------ lifecycle -- */

static void moments(const double *f, double *rho, double *j)
{
    *rho = 0.0;
    j[0] = j[1] = j[2] = 0.0;
    for (int i = 0; i < Q; ++i) {
        *rho += f[i];
        j[0] += CX[i] * f[i];
        j[1] += CY[i] * f[i];
        j[2] += CZ[i] * f[i];
    }
}

static void totals_mass(orc *o)
{
    ksum mc = {0.0, 0.0}, mr = {0.0, 0.0}, mp = {0.0, 0.0};
    for (long n = 0; n < o->n; ++n) {
        if (o->vox[n] != ORC_FLUID)
            continue;
        for (int i = 0; i < Q; ++i) {
            kadd(&mc, o->fC[n * Q + i]);
            kadd(&mr, o->fR[n * Q + i]);
            if (o->fP)
                kadd(&mp, o->fP[n * Q + i]);
        }
    }
    o->tot[0] = kval(&mc);
    o->tot[1] = kval(&mr);
    o->totp[0] = kval(&mp);
}

static void free_all(orc *o)
{
    free(o->vox); free(o->fC); free(o->fR); free(o->pC); free(o->pR); free(o->em); free(o->acc);
    free(o->fP); free(o->pP); free(o->emP); free(o->accP);
    free(o);
}

orc *orc_create(int nx, int ny, int nz, const unsigned char *vox, const orc_params *prm)
{
    if (nx < 1 || ny < 1 || nz < 1 || !vox || !prm)
        return NULL;
    orc *o = calloc(1, sizeof(orc));
    if (!o)
        return NULL;
    o->nx = nx;
    o->ny = ny;
    o->nz = nz;
    o->n = (long)nx * ny * nz;
    o->prm = *prm;
    o->vox = malloc(o->n);
    o->fC = calloc(o->n * Q, sizeof(double));
    o->fR = calloc(o->n * Q, sizeof(double));
    o->pC = calloc(o->n * Q, sizeof(double));
    o->pR = calloc(o->n * Q, sizeof(double));
    o->em = calloc(o->n * Q, sizeof(double));
    o->acc = calloc(o->n, sizeof(double));
    if (prm->product) {
        o->fP = calloc(o->n * Q, sizeof(double));
        o->pP = calloc(o->n * Q, sizeof(double));
        o->emP = calloc(o->n * Q, sizeof(double));
        o->accP = calloc(o->n, sizeof(double));
    }
    if (!o->vox || !o->fC || !o->fR || !o->pC || !o->pR || !o->em || !o->acc ||
        (prm->product && (!o->fP || !o->pP || !o->emP || !o->accP))) {
        free_all(o);
        return NULL;
    }
    memcpy(o->vox, vox, o->n);
    /* Initial state: carrier at rest with density rho0, reactant at c0 (the
     * paper starts with no reactant in the domain), no product (calloc). */
    double zero[3] = {0.0, 0.0, 0.0};
    double eqC[Q], eqR[Q];
    orc_equilibrium(prm->rho0, zero, eqC);
    orc_equilibrium(prm->c0, zero, eqR);
    for (long n = 0; n < o->n; ++n) {
        if (o->vox[n] != ORC_FLUID)
            continue;
        for (int i = 0; i < Q; ++i) {
            o->fC[n * Q + i] = eqC[i];
            o->fR[n * Q + i] = eqR[i];
        }
    }
    totals_mass(o);
    return o;
}

void orc_destroy(orc *o)
{
    if (!o)
        return;
    free_all(o);
}

/* ----------------------------------------------------------------- step -- */

/* Steps 1-4: moments, common velocity, equilibria, BGK collision (plus the
 * forcing term on the carrier), node by node. */
static void collide(orc *o)
{
    const orc_params *P = &o->prm;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < o->nz; ++z) {
        for (int y = 0; y < o->ny; ++y) {
            for (int x = 0; x < o->nx; ++x) {
                long n = node(o, x, y, z);
                if (o->vox[n] != ORC_FLUID)
                    continue;
                const double *fc = o->fC + n * Q, *fr = o->fR + n * Q;
                const double *fp = o->fP ? o->fP + n * Q : NULL;
                double rc, jc[3], rr, jr[3], rp = 0.0, jp[3] = {0.0, 0.0, 0.0}, u[3];
                moments(fc, &rc, jc);
                moments(fr, &rr, jr);
                if (fp)
                    moments(fp, &rp, jp);
                for (int a = 0; a < 3; ++a) {
                    if (P->coupling == ORC_BARYCENTRIC)
                        u[a] = (jc[a] + jr[a] + jp[a] + 0.5 * P->force[a]) / (rc + rr + rp);
                    else
                        u[a] = (jc[a] + 0.5 * P->force[a]) / rc;
                }
                double eqc[Q], eqr[Q], eqp[Q], S[Q];
                orc_equilibrium(rc, u, eqc);
                orc_equilibrium(rr, u, eqr);
                orc_equilibrium(rp, u, eqp);
                orc_guo_source(P->tau_gas, u, P->force, S);
                for (int i = 0; i < Q; ++i) {
                    o->pC[n * Q + i] = fc[i] - (fc[i] - eqc[i]) / P->tau_gas + S[i];
                    o->pR[n * Q + i] = fr[i] - (fr[i] - eqr[i]) / P->tau_species;
                    if (fp)
                        o->pP[n * Q + i] = fp[i] - (fp[i] - eqp[i]) / P->tau_species;
                }
            }
        }
    }
}

/* Philox4x32-10 (Salmon et al. 2011): ten rounds of two 32 x 32 -> 64-bit
 * products, the high halves xored with the other counter words and the key,
 * the key bumped by the Weyl constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3], k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1, n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static int vcode(int i)
{
    return 9 * (CX[i] + 1) + 3 * (CY[i] + 1) + (CZ[i] + 1);
}

/* STOCHASTIC: the exit direction of the arrival at node k along active link
 * j produced by the collision of step t (see the header). */
static int random_exit(const orc *o, long k, int j, unsigned act, int b, long t)
{
    int exits[Q], n = 0;
    for (int code = 0; code < 27; ++code)
        for (int e = 1; e < Q; ++e)
            if (vcode(e) == code && (act & (1u << OPP[e])))
                exits[n++] = e;
    uint32_t ctr[4] = {(uint32_t)t, (uint32_t)k, (uint32_t)vcode(j), 0u};
    uint32_t key[2] = {(uint32_t)o->prm.seed, (uint32_t)(o->prm.seed >> 32)}, out[4];
    orc_philox4x32_10(ctr, key, out);
    (void)n;
    return exits[(int)(((uint64_t)out[0] * (uint64_t)b) >> 32)];
}

/* Step 5: the sputtering boundary condition at catalytic nodes.  Returns the
 * total reactant arrival sum_k In_R(k) of this step, and the product arrival
 * sum_k In_P(k) in *arrived_p (0 without the product lattice). */
static double interface(orc *o, double *arrived_p)
{
    const orc_params *P = &o->prm;
    int xper = P->species_x == ORC_XPERIODIC;
    ksum total = {0.0, 0.0}, total_p = {0.0, 0.0};
    for (int z = 0; z < o->nz; ++z)
        for (int y = 0; y < o->ny; ++y)
            for (int x = 0; x < o->nx; ++x) {
                long k = node(o, x, y, z);
                if (o->vox[k] != ORC_CATALYTIC)
                    continue;
                unsigned act;
                int b = active_links(o, x, y, z, &act);
                if (b == 0)
                    continue;
                /* In(k): every reactant population heading into k along an
                 * active link, f*_j(k - c_j). */
                double in = 0.0, in_p = 0.0, wsum = 0.0;
                for (int j = 1; j < Q; ++j) {
                    if (!(act & (1u << j)))
                        continue;
                    int sx, sy, sz;
                    source(o, x, y, z, j, xper, &sx, &sy, &sz);
                    in += o->pR[node(o, sx, sy, sz) * Q + j];
                    if (o->pP)
                        in_p += o->pP[node(o, sx, sy, sz) * Q + j];
                    wsum += WT[OPP[j]];
                }
                o->acc[k] += in;
                kadd(&total, in);
                if (o->pP) {
                    o->accP[k] += in_p;
                    kadd(&total_p, in_p);
                }
                /* What the node sends back as product: the converted part of
                 * the reactant plus the product that did not stick. */
                const double a_r = P->p * P->p_stick, a_p = 1.0 - P->p_stick_product;
                if (P->sputter == ORC_STOCHASTIC) {
                    /* each arrival leaves whole along one random exit */
                    for (int i = 0; i < Q; ++i) {
                        o->em[k * Q + i] = 0.0;
                        if (o->emP)
                            o->emP[k * Q + i] = 0.0;
                    }
                    for (int j = 1; j < Q; ++j) {
                        if (!(act & (1u << j)))
                            continue;
                        int sx, sy, sz;
                        source(o, x, y, z, j, xper, &sx, &sy, &sz);
                        long s = node(o, sx, sy, sz);
                        int e = random_exit(o, k, j, act, b, o->step);
                        o->em[k * Q + e] += (1.0 - P->p_stick) * o->pR[s * Q + j];
                        if (o->emP)
                            o->emP[k * Q + e] += a_r * o->pR[s * Q + j] + a_p * o->pP[s * Q + j];
                    }
                    continue;
                }
                /* Re-emission (1 - p_S^R) sum_j S_ij f_j^out along i = opp(j). */
                for (int j = 1; j < Q; ++j) {
                    if (!(act & (1u << j)))
                        continue;
                    int i = OPP[j];
                    double e, ep;
                    if (P->sputter == ORC_UNIFORM) {
                        e = (1.0 - P->p_stick) * in / b;
                        ep = (a_r * in + a_p * in_p) / b;
                    } else if (P->sputter == ORC_WEIGHTED) {
                        e = (1.0 - P->p_stick) * in * WT[i] / wsum;
                        ep = (a_r * in + a_p * in_p) * WT[i] / wsum;
                    } else {
                        int sx, sy, sz;
                        source(o, x, y, z, j, xper, &sx, &sy, &sz);
                        long s = node(o, sx, sy, sz);
                        e = (1.0 - P->p_stick) * o->pR[s * Q + j];
                        ep = a_r * o->pR[s * Q + j] + (o->pP ? a_p * o->pP[s * Q + j] : 0.0);
                    }
                    o->em[k * Q + i] = e;
                    if (o->emP)
                        o->emP[k * Q + i] = ep;
                }
            }
    *arrived_p = kval(&total_p);
    return kval(&total);
}

/* Pull of one species lattice into gas node (x, y, z): post-collision
 * populations pst, catalytic emission em, inlet ghost values ghost[i]. */
static void pull_species(orc *o, int x, int y, int z, const double *pst, const double *em,
                         const double *ghost, double *f)
{
    int res = o->prm.species_x != ORC_XPERIODIC;
    long n = node(o, x, y, z);
    for (int i = 0; i < Q; ++i) {
        int sx, sy, sz;
        long s;
        source(o, x, y, z, i, !res, &sx, &sy, &sz);
        double v;
        if (sx < 0) {
            v = ghost[i];                                    /* inlet ghost */
        } else if (sx >= o->nx) {
            long m = node(o, o->nx - 1, sy, sz);             /* outlet ghost */
            v = o->vox[m] == ORC_FLUID ? pst[m * Q + i] : pst[n * Q + OPP[i]];
        } else {
            s = node(o, sx, sy, sz);
            if (o->vox[s] == ORC_FLUID)
                v = pst[s * Q + i];
            else if (o->vox[s] == ORC_INERT)
                v = pst[n * Q + OPP[i]];
            else
                v = em[s * Q + i];
        }
        f[n * Q + i] = v;
    }
}

/* Step 6: pull streaming of every lattice. */
static void stream(orc *o)
{
    const orc_params *P = &o->prm;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < o->nz; ++z) {
        for (int y = 0; y < o->ny; ++y) {
            for (int x = 0; x < o->nx; ++x) {
                long n = node(o, x, y, z);
                if (o->vox[n] != ORC_FLUID)
                    continue;
                double M = 0.0, W = 0.0;
                for (int i = 0; i < Q; ++i) {
                    int sx, sy, sz;
                    /* carrier: periodic in x; every solid reflects */
                    source(o, x, y, z, i, 1, &sx, &sy, &sz);
                    long s = node(o, sx, sy, sz);
                    o->fC[n * Q + i] = o->vox[s] == ORC_FLUID ? o->pC[s * Q + i] : o->pC[n * Q + OPP[i]];
                    if (o->vox[s] != ORC_FLUID) {
                        M += o->pC[n * Q + OPP[i]];
                        W += WT[i];
                    }
                }
                if (P->wall_diffuse != 0.0 && W > 0.0)
                    for (int i = 0; i < Q; ++i) {
                        int sx, sy, sz;
                        source(o, x, y, z, i, 1, &sx, &sy, &sz);
                        if (o->vox[node(o, sx, sy, sz)] != ORC_FLUID)
                            o->fC[n * Q + i] = (1.0 - P->wall_diffuse) * o->pC[n * Q + OPP[i]] +
                                               P->wall_diffuse * WT[i] * M / W;
                    }
                /* the inlet ghost of INFLOW moves with the carrier velocity of this node */
                double ghost[Q];
                for (int i = 0; i < Q; ++i)
                    ghost[i] = WT[i] * P->c_inlet;
                if (P->species_x == ORC_XINFLOW && x == 0) {
                    double rho, j[3], u[3];
                    moments(o->fC + n * Q, &rho, j);
                    for (int d = 0; d < 3; ++d)
                        u[d] = (j[d] + 0.5 * P->force[d]) / rho;
                    orc_equilibrium(P->c_inlet, u, ghost);
                }
                pull_species(o, x, y, z, o->pR, o->em, ghost, o->fR);
                if (o->fP) {
                    double none[Q] = {0.0};                              /* no product is injected */
                    pull_species(o, x, y, z, o->pP, o->emP, none, o->fP);
                }
            }
        }
    }
}

/* A species crossing the x-boundaries during the streaming just done: in_flux
 * pulled from the inlet ghost; out_in left through the inlet face; out_out
 * sent to the outlet ghost net of what it returned.  f / pst: pre- and
 * post-collision populations of that species. */
static void boundary_flux(orc *o, const double *f, const double *pst, double *in_flux, double *out_in,
                          double *out_out)
{
    ksum fin = {0.0, 0.0}, foi = {0.0, 0.0}, foo = {0.0, 0.0};
    *in_flux = 0.0;
    *out_in = 0.0;
    *out_out = 0.0;
    if (o->prm.species_x == ORC_XPERIODIC)
        return;
    for (int z = 0; z < o->nz; ++z)
        for (int y = 0; y < o->ny; ++y) {
            long n0 = node(o, 0, y, z);
            if (o->vox[n0] == ORC_FLUID)
                for (int i = 1; i < Q; ++i) {
                    if (CX[i] == 1)
                        kadd(&fin, f[n0 * Q + i]);                 /* pulled from the inlet ghost */
                    if (CX[i] == -1)
                        kadd(&foi, pst[n0 * Q + i]);              /* left through the inlet */
                }
            long n1 = node(o, o->nx - 1, y, z);
            if (o->vox[n1] == ORC_FLUID)
                for (int i = 1; i < Q; ++i) {
                    if (CX[i] == 1)
                        kadd(&foo, pst[n1 * Q + i]);              /* sent to the outlet ghost */
                    if (CX[i] == -1)
                        kadd(&foo, -f[n1 * Q + i]);               /* came back from it */
                }
        }
    *in_flux = kval(&fin);
    *out_in = kval(&foi);
    *out_out = kval(&foo);
}

void orc_step(orc *o, long nsteps)
{
    const orc_params *P = &o->prm;
    for (long t = 0; t < nsteps; ++t) {
        collide(o);
        double arrived_p;
        double arrived = interface(o, &arrived_p);
        stream(o);
        double fin, foi, foo;
        boundary_flux(o, o->fR, o->pR, &fin, &foi, &foo);
        totals_mass(o);
        o->tot[2] += P->p * P->p_stick * arrived;
        o->tot[3] += (1.0 - P->p) * P->p_stick * arrived;
        o->tot[4] += fin;
        o->tot[5] += foi + foo;
        if (o->fP) {
            double pin;
            boundary_flux(o, o->fP, o->pP, &pin, &foi, &foo);
            o->totp[1] += P->p_stick_product * arrived_p;
            o->totp[2] += foi;
            o->totp[3] += foo;
        }
        o->step += 1;
    }
}

/* ------------------------------------------------------------- outputs -- */

/* Moments of the pre-collision populations at the current step; solid 0.
 * u is component-major (u[a * n + node]). */
void orc_fields(const orc *o, double *rho, double *u, double *conc)
{
    const orc_params *P = &o->prm;
    for (long n = 0; n < o->n; ++n) {
        double rc = 0.0, jc[3] = {0, 0, 0}, rr = 0.0, jr[3] = {0, 0, 0}, v[3] = {0, 0, 0};
        double rp = 0.0, jp[3] = {0, 0, 0};
        if (o->vox[n] == ORC_FLUID) {
            moments(o->fC + n * Q, &rc, jc);
            moments(o->fR + n * Q, &rr, jr);
            if (o->fP)
                moments(o->fP + n * Q, &rp, jp);
            for (int a = 0; a < 3; ++a) {
                if (P->coupling == ORC_BARYCENTRIC)
                    v[a] = (jc[a] + jr[a] + jp[a] + 0.5 * P->force[a]) / (rc + rr + rp);
                else
                    v[a] = (jc[a] + 0.5 * P->force[a]) / rc;
            }
        }
        if (rho) rho[n] = rc;
        if (conc) conc[n] = rr;
        if (u)
            for (int a = 0; a < 3; ++a)
                u[a * o->n + n] = v[a];
    }
}

/* Converted reactant per voxel: p p_S^R sum_t In(k, t) at catalytic nodes. */
void orc_conversion_map(const orc *o, double *conv)
{
    for (long n = 0; n < o->n; ++n)
        conv[n] = o->vox[n] == ORC_CATALYTIC ? o->prm.p * o->prm.p_stick * o->acc[n] : 0.0;
}

void orc_totals(const orc *o, double *t)
{
    for (int k = 0; k < 6; ++k)
        t[k] = o->tot[k];
}

/* Product diagnostics (zeros without the product lattice): conc[node] =
 * rho_P of the pre-collision populations (solid 0); tot = {mass_product,
 * lost_product, product out through the inlet face, product out through the
 * outlet face}; conv_p[node] = p_S^P sum_t In_P(k, t), the product that stuck
 * at catalytic node k. */
void orc_product(const orc *o, double *conc, double *tot, double *stuck)
{
    for (long n = 0; n < o->n; ++n) {
        double r = 0.0;
        if (o->fP && o->vox[n] == ORC_FLUID)
            for (int i = 0; i < Q; ++i)
                r += o->fP[n * Q + i];
        if (conc) conc[n] = r;
        if (stuck)
            stuck[n] = o->accP && o->vox[n] == ORC_CATALYTIC ? o->prm.p_stick_product * o->accP[n] : 0.0;
    }
    if (tot)
        for (int k = 0; k < 4; ++k)
            tot[k] = o->fP ? o->totp[k] : 0.0;
}

/* Product flux profile along the flow (Eq. for Phi_P, with x the streamwise
 * axis here): phi[x] = sum over the (y, z) cross-section of rho_P u_x, the
 * moments of the pre-collision populations, u the species advection
 * velocity. */
void orc_product_flux(const orc *o, double *phi)
{
    const orc_params *P = &o->prm;
    for (int x = 0; x < o->nx; ++x) {
        ksum s = {0.0, 0.0};
        if (o->fP)
            for (int z = 0; z < o->nz; ++z)
                for (int y = 0; y < o->ny; ++y) {
                    long n = node(o, x, y, z);
                    if (o->vox[n] != ORC_FLUID)
                        continue;
                    double rc, jc[3], rr, jr[3], rp, jp[3], ux;
                    moments(o->fC + n * Q, &rc, jc);
                    moments(o->fR + n * Q, &rr, jr);
                    moments(o->fP + n * Q, &rp, jp);
                    if (P->coupling == ORC_BARYCENTRIC)
                        ux = (jc[0] + jr[0] + jp[0] + 0.5 * P->force[0]) / (rc + rr + rp);
                    else
                        ux = (jc[0] + 0.5 * P->force[0]) / rc;
                    kadd(&s, rp * ux);
                }
        phi[x] = kval(&s);
    }
}

long orc_step_count(const orc *o)
{
    return o->step;
}

/* Direct access to the pre-collision state, for closed-form tests. */
void orc_get_state(const orc *o, double *fC, double *fR)
{
    if (fC) memcpy(fC, o->fC, sizeof(double) * o->n * Q);
    if (fR) memcpy(fR, o->fR, sizeof(double) * o->n * Q);
}

void orc_set_state(orc *o, const double *fC, const double *fR)
{
    if (fC) memcpy(o->fC, fC, sizeof(double) * o->n * Q);
    if (fR) memcpy(o->fR, fR, sizeof(double) * o->n * Q);
    totals_mass(o);
}

/* The same for the product lattice (no-ops without it). */
void orc_get_state_product(const orc *o, double *fP)
{
    if (fP && o->fP) memcpy(fP, o->fP, sizeof(double) * o->n * Q);
}

void orc_set_state_product(orc *o, const double *fP)
{
    if (fP && o->fP) memcpy(o->fP, fP, sizeof(double) * o->n * Q);
    totals_mass(o);
}

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the next parallel regions (for timing single-thread and
 * all-core runs); results do not depend on it. */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}
