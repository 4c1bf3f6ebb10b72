// C ABI of the reactive lattice-Boltzmann library (declared in include/lbm.h):
// argument checking, the create-time preprocessing of the voxel map (chunk
// records and the compacted interface list), device memory, the step loop
// and the outputs.  All per-step arithmetic runs in the HIP kernels.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm2d.h"
#include "lbm_internal.h"

using namespace lbmk;

namespace {

thread_local std::string g_create_error;

constexpr double CS = 0.57735026918962576451;  // lattice sound speed 1/sqrt(3)
constexpr int TIMING_RING = 512;
constexpr uint64_t CKPT_MAGIC = 0x3847504b434d424cull;  // "LBMCKPG8"

struct StepEvents {
    hipEvent_t ev[8];  // start/stop of the front launch, xflux, sweep, closing reduction
    bool pending;
    bool flushed;      // the slot's step closed an lbm_step call (ev[6..7] time that reduction)
    bool sweep_only;   // only ev[4..5] were recorded
};

uint64_t fnv1a(const uint8_t *p, size_t n) {
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

}  // namespace

struct lbm_ctx {
    // sizes and parameters
    int nx = 0, ny = 0, nz = 0, W = 0;
    int64_t n = 0, nfluid = 0, nfp = 0, niface = 0, nlinks = 0;
    uint32_t lay_ss = 0, lay_bs = 0;  // population layout (Geometry::lay_ss / lay_bs)
    double kn = 0, da = 0, delta = 0, p = 0;
    int p_clamped = 0;
    int wall_clamped = 0;  // the Kn relation clamped the wall's diffuse fraction
    int lattice = LBM_LATTICE_D3Q19;
    lbm2d::Dev d2{};       // device state of a D2Q9 context
    Physics ph{};
    std::vector<uint8_t> vox;
    std::vector<uint32_t> iface_vox;  // host copy for the conversion map
    uint64_t geom_hash = 0;
    std::string err;

    // device
    lbm_device dev{};
    hipStream_t stream = nullptr;
    int64_t device_bytes = 0;
    std::vector<void *> allocations;
    ChunkInfo *d_chunks = nullptr;
    uint32_t *d_order = nullptr;
    uint32_t *d_iface_vox = nullptr, *d_iface_mask = nullptr;
    double *d_iface_scale = nullptr, *d_acc = nullptr;
    unsigned long long *d_inacc = nullptr;  // In(k) of the sweep in progress (fixed point)
    void *d_emit = nullptr;
    void *d_pop[2] = {nullptr, nullptr};
    double *d_part = nullptr;
    DevTotals *d_tot = nullptr;
    int device = 0;       // the HIP device the context was created on
    int cur = 0;          // d_pop[cur] holds the post-collision state of the current step
    int64_t step = 0;
    int64_t blocks_sweep = 0, blocks_iface = 0;
    int64_t part_rows = 0;    // sweep-partial rows reserved in d_part (the larger sweep variant's blocks)
    int ytile = 16;       // rows per y-tile of the sweep traversal
    // node-compact sweep: per-node coordinates and wave launch order;
    // compact = 1 selects it (needs ny, nz <= 1024)
    uint32_t *d_pos = nullptr, *d_worder = nullptr, *d_wunits = nullptr;
    int64_t nwaves = 0;
    bool compact_ok = false;
    int compact = 0;

    // product lattice (ph.product): populations (same parity as d_pop), E_P,
    // In_P, Acc_P and partial sums (3 per sweep block, then 2 x interface)
    void *d_popP[2] = {nullptr, nullptr};
    void *d_emitP = nullptr;
    unsigned long long *d_inaccP = nullptr;
    double *d_accP = nullptr;
    double *d_partP = nullptr;
    int64_t rows_partP = 0;   // sweep-partial rows reserved in d_partP

    // watchdog
    int32_t *h_flag = nullptr;
    hipEvent_t flag_event = nullptr;
    bool flag_pending = false;

    // timing
    int timing = 0;  // 0 off, 1 every launch, 2 the sweep only
    std::vector<StepEvents> ring;
    int ring_next = 0;
    lbm_kernel_times_t times{};
};

namespace {

// Temporary device memory through the context's allocator (defined below).
void *scratch_alloc(lbm_ctx *c, size_t bytes);
void scratch_free(lbm_ctx *c, void *p);

lbm_status fail(lbm_ctx *c, lbm_status s, const std::string &msg) {
    if (c)
        c->err = msg;
    else
        g_create_error = msg;
    return s;
}

lbm_status hip_fail(lbm_ctx *c, hipError_t e, const char *what) {
    return fail(c, e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

void *dev_alloc(lbm_ctx *c, size_t bytes) {
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (c->dev.alloc) {
        p = c->dev.alloc(bytes, c->dev.user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) {
        c->allocations.push_back(p);
        c->device_bytes += int64_t(bytes);
    }
    return p;
}

void release(lbm_ctx *c) {
    for (void *p : c->allocations) {
        if (c->dev.free)
            c->dev.free(p, c->dev.user);
        else
            (void)hipFree(p);
    }
    c->allocations.clear();
    for (auto &r : c->ring)
        for (auto &e : r.ev) (void)hipEventDestroy(e);
    c->ring.clear();
    if (c->flag_event) (void)hipEventDestroy(c->flag_event);
    if (c->h_flag) (void)hipHostFree(c->h_flag);
}

Geometry geometry(const lbm_ctx *c) {
    Geometry g;
    g.chunks = c->d_chunks;
    g.order = c->d_order;
    g.inacc = c->d_inacc;
    g.nx = c->nx;
    g.ny = c->ny;
    g.nz = c->nz;
    g.W = c->W;
    g.units = uint32_t(int64_t(c->ny) * c->nz * c->W);
    g.niface = uint32_t(c->niface);
    g.nfp = c->nfp;
    g.lay_ss = c->lay_ss;
    g.lay_bs = c->lay_bs;
    g.nfluid = c->nfluid;
    g.pos = c->d_pos;
    g.worder = c->d_worder;
    g.wunits = c->d_wunits;
    g.nwaves = uint32_t(c->nwaves);
    g.pad2 = 0;
    g.inv_W = 1.0 / double(c->W);
    g.inv_ny = 1.0 / double(c->ny);
    g.ivox = c->d_iface_vox;
    g.imask = c->d_iface_mask;
    return g;
}

// In and emission slots per interface node: one, or one per exit direction
// for STOCHASTIC.
int64_t nslot(const lbm_ctx *c) { return c->ph.sputter == SP_STOCHASTIC ? NSLOT : 1; }

// Sweep blocks of the variant in use (the partial sums have one row each).
int64_t active_sweep_blocks(const lbm_ctx *c) {
    return c->compact ? sweep_blocks_c(geometry(c)) : c->blocks_sweep;
}

// Per compact wave w: the (row, chunk) unit of its first node, u0 = (z ny +
// y) W + x / 64, and the number of consecutive units its 64 nodes span
// (capped at 63), as u0 | nu << 26 (u0 < 2^26 since ny, nz <= 1024 and
// W <= 64).  The sweep loads its wavefront's records cooperatively when nu is
// small, and finds each lane's coordinates from them.
void build_wave_units(const lbm_ctx *c, const std::vector<uint32_t> &pos, std::vector<uint32_t> &wunits) {
    auto unit = [&](uint32_t p) {
        const uint32_t x = p & 0xfffu, y = (p >> 12) & 0x3ffu, z = p >> 22;
        return (z * uint32_t(c->ny) + y) * uint32_t(c->W) + (x >> 6);
    };
    wunits.resize(size_t(c->nwaves));
    for (int64_t w = 0; w < c->nwaves; ++w) {
        const int64_t last = std::min<int64_t>(c->nfluid, w * 64 + 64) - 1;
        const uint32_t u0 = unit(pos[size_t(w * 64)]), u1 = unit(pos[size_t(last)]);
        wunits[size_t(w)] = u0 | (std::min<uint32_t>(u1 - u0 + 1u, 63u) << 26);
    }
}

// Launch order of the node-compact waves: wave w (storage indices 64 w ..)
// goes with the row of its first node, rows in the y-tiled order of
// build_order, waves of one row in storage order.
void build_wave_order(const lbm_ctx *c, const std::vector<uint32_t> &pos, int ytile, std::vector<uint32_t> &worder) {
    std::vector<uint32_t> order(size_t(int64_t(c->ny) * c->nz * c->W));
    build_order(c->nx, c->ny, c->nz, ytile, order.data());
    std::vector<uint32_t> row_seq(size_t(int64_t(c->ny) * c->nz), 0);
    uint32_t seq = 0;
    for (uint32_t code : order) {
        if ((code >> 24) != 0) continue;  // first chunk of each row
        const uint32_t y = code & 0xfffu, z = (code >> 12) & 0xfffu;
        row_seq[size_t(z) * c->ny + y] = seq++;
    }
    std::vector<uint64_t> key(size_t(c->nwaves));
    for (int64_t w = 0; w < c->nwaves; ++w) {
        const uint32_t p = pos[size_t(w * 64)];
        const uint32_t y = (p >> 12) & 0x3ffu, z = p >> 22;
        key[size_t(w)] = (uint64_t(row_seq[size_t(z) * c->ny + y]) << 32) | uint64_t(w);
    }
    std::sort(key.begin(), key.end());
    worder.resize(size_t(c->nwaves));
    for (size_t k = 0; k < key.size(); ++k) worder[k] = uint32_t(key[k] & 0xffffffffu);
}

Interface interface_list(const lbm_ctx *c) {
    Interface it;
    it.vox = c->d_iface_vox;
    it.mask = c->d_iface_mask;
    it.scale = c->d_iface_scale;
    it.acc = c->d_acc;
    it.inacc = c->d_inacc;
    it.n = c->niface;
    return it;
}

// Chunk records of every x-row: gas/catalytic bits, storage base, and the
// periodic left/right neighbours of the chunk.
void build_chunks(const lbm_ctx *c, const std::vector<uint32_t> &ivox, std::vector<ChunkInfo> &ch) {
    const int64_t rows = int64_t(c->ny) * c->nz;
    ch.assign(size_t(rows * c->W), ChunkInfo{});
    std::vector<uint8_t> is_iface(size_t(c->n), 0);
    for (uint32_t v : ivox) is_iface[v] = 1;
    uint64_t running = 0, irunning = 0;
    for (int64_t r = 0; r < rows; ++r) {
        const uint8_t *v = c->vox.data() + r * c->nx;
        const uint8_t *f = is_iface.data() + r * c->nx;
        for (int k = 0; k < c->W; ++k) {
            ChunkInfo &I = ch[size_t(r * c->W + k)];
            for (int b = 0; b < 64; ++b) {
                const int x = 64 * k + b;
                if (x >= c->nx) break;
                if (v[x] == LBM_FLUID) I.fluid |= 1ull << b;
                if (f[x]) I.cat |= 1ull << b;
            }
            I.base = uint32_t(running);
            I.ibase = uint32_t(irunning);
            running += uint64_t(__builtin_popcountll(I.fluid));
            irunning += uint64_t(__builtin_popcountll(I.cat));
        }
    }
    // periodic x-neighbours of each chunk: storage index when gas, interface
    // index when an interface node
    auto neighbour = [&](int64_t r, int x) -> uint32_t {
        const ChunkInfo &I = ch[size_t(r * c->W + (x >> 6))];
        const int b = x & 63;
        const uint64_t below = b ? (~0ull >> (64 - b)) : 0ull;
        if ((I.fluid >> b) & 1u) return NB_GAS | (I.base + uint32_t(__builtin_popcountll(I.fluid & below)));
        if ((I.cat >> b) & 1u) return NB_CAT | (I.ibase + uint32_t(__builtin_popcountll(I.cat & below)));
        return 0u;
    };
    for (int64_t r = 0; r < rows; ++r) {
        for (int k = 0; k < c->W; ++k) {
            ChunkInfo &I = ch[size_t(r * c->W + k)];
            const int xp = k > 0 ? 64 * k - 1 : c->nx - 1;
            const int xn = 64 * k + 64 < c->nx ? 64 * k + 64 : 0;
            I.prev = neighbour(r, xp);
            I.next = neighbour(r, xn);
        }
    }
}

// Interface list: catalytic nodes with at least one active link (a link j
// whose pull source k - c_j is a gas node inside the domain).
void build_interface(lbm_ctx *c, std::vector<uint32_t> &vox, std::vector<uint32_t> &mask,
                     std::vector<double> &scale) {
    const bool xper = c->ph.species_x == XB_PERIODIC;
    c->nlinks = 0;
    for (int z = 0; z < c->nz; ++z)
        for (int y = 0; y < c->ny; ++y)
            for (int x = 0; x < c->nx; ++x) {
                const int64_t k = (int64_t(z) * c->ny + y) * c->nx + x;
                if (c->vox[size_t(k)] != LBM_CATALYTIC) continue;
                uint32_t m = 0;
                int b = 0;
                double wsum = 0.0;
                for (int j = 1; j < 19; ++j) {
                    int xs = x - CX[j];
                    const int ys = (y - CY[j] + c->ny) % c->ny, zs = (z - CZ[j] + c->nz) % c->nz;
                    if (xs < 0 || xs >= c->nx) {
                        if (!xper) continue;
                        xs = (xs + c->nx) % c->nx;
                    }
                    if (c->vox[size_t((int64_t(zs) * c->ny + ys) * c->nx + xs)] == LBM_FLUID) {
                        m |= 1u << j;
                        ++b;
                        wsum += wgt<double>(opp(j));
                    }
                }
                if (b == 0) continue;
                vox.push_back(uint32_t(k));
                mask.push_back(m);
                scale.push_back(c->ph.sputter == SP_WEIGHTED ? 1.0 / wsum : 1.0 / b);
                c->nlinks += b;
            }
}


lbm_status check_pending_flag(lbm_ctx *c) {
    if (c->flag_pending && hipEventQuery(c->flag_event) == hipSuccess) {
        c->flag_pending = false;
        if (*c->h_flag) return fail(c, LBM_ENONFINITE, "a global total became non-finite");
    }
    return LBM_OK;
}

void drain_slot(lbm_ctx *c, StepEvents &r) {
    if (!r.pending) return;
    (void)hipEventSynchronize(r.ev[r.sweep_only ? 5 : 7]);
    float ms[4];
    for (int k = 0; k < 4; ++k) {
        ms[k] = 0.0f;
        if ((!r.sweep_only || k == 2) && hipEventElapsedTime(&ms[k], r.ev[2 * k], r.ev[2 * k + 1]) != hipSuccess)
            ms[k] = 0.0f;
    }
    if (c->blocks_iface > 0 && !r.sweep_only) {
        c->times.ms_interface += ms[0];
        c->times.n_interface += 1;
    }
    c->times.ms_sweep += ms[2];
    c->times.n_sweep += 1;
    if (r.flushed && !r.sweep_only) {
        c->times.ms_reduce += ms[3];
        c->times.n_reduce += 1;
    }
    r.pending = false;
}

// Partial-sum layout in d_part: sweep partials (4 per sweep block), then the
// interface partials and the fold outputs, two of each alternating with the
// step's parity (a front launch writes step t's while it reads step t - 1's).
double *part_iface(const lbm_ctx *c, int64_t t) { return c->d_part + 4 * c->part_rows + (t & 1) * c->blocks_iface; }
double *part_fold(const lbm_ctx *c, int64_t t) {
    return c->d_part + 4 * c->part_rows + 2 * c->blocks_iface + (t & 1) * int64_t(FOLD_BLOCKS) * NPART;
}
double *part_iface_p(const lbm_ctx *c, int64_t t) {
    return c->d_partP + 3 * c->rows_partP + (t & 1) * c->blocks_iface;
}

// The product lattice's buffers for step t (reading d_popP[cur]).
ProdStep prod_step(const lbm_ctx *c, int64_t t) {
    ProdStep p{};
    p.fin = c->d_popP[c->cur];
    p.fout = c->d_popP[1 - c->cur];
    p.emit = c->d_emitP;
    p.inacc = c->d_inaccP;
    p.acc = c->d_accP;
    p.part_sweep = c->d_partP;
    p.pi_now = part_iface_p(c, t);
    p.pi_prev = part_iface_p(c, t - 1);
    return p;
}

// One step t = c->step: the front launch (interface of t, and the reduction
// stages of t - 1 and t - 2 when those steps belong to the same lbm_step
// call: `fold`, `reduce`), then the sweep.  `last` closes the call: the
// remaining reduction stages of t - 1 and t follow the sweep.
lbm_status one_step(lbm_ctx *c, bool fold, bool reduce, bool last) {
    const Geometry g = geometry(c);
    const void *fin = c->d_pop[c->cur];
    void *fout = c->d_pop[1 - c->cur];
    const int64_t t = c->step;
    double *ps = c->d_part;
    const int64_t ns = active_sweep_blocks(c), ni = c->blocks_iface;
    StepEvents *r = nullptr, *all = nullptr;  // all: every launch is timed
    if (c->timing) {
        r = &c->ring[size_t(c->ring_next)];
        c->ring_next = (c->ring_next + 1) % TIMING_RING;
        drain_slot(c, *r);
        if (c->timing == 1) all = r;
    }
    hipError_t e;
    ProdStep pst = c->ph.product ? prod_step(c, t) : ProdStep{};
    const ProdStep *prod = c->ph.product ? &pst : nullptr;
    if (all) (void)hipEventRecord(r->ev[0], c->stream);
    e = launch_front(c->ph, interface_list(c), c->d_emit, c->blocks_iface, part_iface(c, t), ps, ns,
                     part_iface(c, t - 1), ni, part_fold(c, t - 1), fold, part_fold(c, t - 2), reduce, c->d_tot,
                     c->stream, prod);
    if (e != hipSuccess) return hip_fail(c, e, "interface kernel launch");
    if (all) (void)hipEventRecord(r->ev[1], c->stream);
    if (all) (void)hipEventRecord(r->ev[2], c->stream);  // no separate boundary-flux kernel:
    if (all) (void)hipEventRecord(r->ev[3], c->stream);  // the sweep tallies the x-planes
    if (r) (void)hipEventRecord(r->ev[4], c->stream);
    c->ph.step_ctr = uint32_t(t + 1);  // this sweep's collision makes the arrivals of step t + 1
    e = c->compact ? launch_sweep_c(g, c->ph, fin, fout, c->d_emit, ps, c->stream, prod)
                   : launch_sweep(g, c->ph, fin, fout, c->d_emit, ps, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "sweep kernel launch");
    if (r) (void)hipEventRecord(r->ev[5], c->stream);
    if (all) (void)hipEventRecord(r->ev[6], c->stream);
    if (last) {
        // fold of t (with the final stage of t - 1 when pending), then the final stage of t
        // (the product partials of step t: the interface ones were written
        // by this step's front launch, as pi_now)
        if (prod) pst.pi_prev = pst.pi_now;
        e = launch_front(c->ph, interface_list(c), c->d_emit, 0, nullptr, ps, ns, part_iface(c, t), ni,
                         part_fold(c, t), true, part_fold(c, t - 1), fold, c->d_tot, c->stream, prod);
        if (e == hipSuccess)
            e = launch_front(c->ph, interface_list(c), c->d_emit, 0, nullptr, ps, ns, nullptr, ni, nullptr, false,
                             part_fold(c, t), true, c->d_tot, c->stream, prod);
        if (e != hipSuccess) return hip_fail(c, e, "reduce kernel launch");
    }
    if (r) {
        if (all) (void)hipEventRecord(r->ev[7], c->stream);
        r->pending = true;
        r->flushed = last;
        r->sweep_only = !all;
    }
    c->cur = 1 - c->cur;
    c->step += 1;
    return LBM_OK;
}

lbm_status validate(const lbm_geometry *g, double kn, double da, const double tau[2], const lbm_bc *bc,
                    lbm_ctx **out) {
    if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!g || !bc || !tau) return fail(nullptr, LBM_EINVAL, "geometry, tau and bc must not be NULL");
    if (!g->voxels) return fail(nullptr, LBM_EINVAL, "geometry voxels is NULL");
    if (g->nx < 1 || g->ny < 1 || g->nz < 1) return fail(nullptr, LBM_EINVAL, "lattice sizes must be >= 1");
    if (g->nx > 4096 || g->ny > 4096 || g->nz > 4096)
        return fail(nullptr, LBM_EINVAL, "nx, ny and nz must be <= 4096");
    if (int64_t(g->nx) * g->ny * g->nz >= (int64_t(1) << 32))
        return fail(nullptr, LBM_EINVAL, "lattice has 2^32 nodes or more");
    if (g->reserved0 != 0) return fail(nullptr, LBM_EINVAL, "reserved fields must be 0");
    if (bc->rounding != LBM_ROUND_NEAREST && bc->rounding != LBM_ROUND_STOCHASTIC)
        return fail(nullptr, LBM_EINVAL, "rounding must be LBM_ROUND_NEAREST or LBM_ROUND_STOCHASTIC");
    if (bc->product != 0 && bc->product != 1) return fail(nullptr, LBM_EINVAL, "product must be 0 or 1");
    if (bc->product && !(bc->p_stick_product >= 0.0 && bc->p_stick_product <= 1.0))
        return fail(nullptr, LBM_EINVAL, "p_stick_product must be in [0, 1]");
    if (bc->product && bc->coupling != LBM_COUPLE_PASSIVE)
        return fail(nullptr, LBM_EUNSUPPORTED, "the product lattice needs PASSIVE coupling");
    if (!(g->pore_size > 0) || !std::isfinite(g->pore_size))
        return fail(nullptr, LBM_EINVAL, "pore_size must be finite and > 0");
    if (bc->sputter < 0 || bc->sputter > 3) return fail(nullptr, LBM_EUNSUPPORTED, "unknown sputter mode");
    if (!(bc->wall_diffuse >= 0.0 && bc->wall_diffuse <= 1.0))
        return fail(nullptr, LBM_EINVAL, "wall_diffuse must be in [0, 1]");
    if (!(bc->wall_accommodation >= 0.0 && bc->wall_accommodation <= 1.0))
        return fail(nullptr, LBM_EINVAL, "wall_accommodation must be in [0, 1]");
    if (bc->wall_accommodation > 0.0 && bc->wall_diffuse != 0.0)
        return fail(nullptr, LBM_EINVAL, "give wall_diffuse or wall_accommodation, not both");
    if (bc->reserved_bc != 0) return fail(nullptr, LBM_EINVAL, "reserved fields must be 0");
    if (bc->lattice != LBM_LATTICE_D3Q19 && bc->lattice != LBM_LATTICE_D2Q9)
        return fail(nullptr, LBM_EINVAL, "lattice must be LBM_LATTICE_D3Q19 or LBM_LATTICE_D2Q9");
    if (bc->lattice == LBM_LATTICE_D2Q9) {
        if (g->nz != 1) return fail(nullptr, LBM_EINVAL, "D2Q9 runs on one plane (nz = 1)");
        if (bc->storage != LBM_STORE_F64) return fail(nullptr, LBM_EUNSUPPORTED, "D2Q9 runs in FP64 storage only");
        if (bc->sputter == LBM_SPUTTER_STOCHASTIC)
            return fail(nullptr, LBM_EUNSUPPORTED, "STOCHASTIC sputtering is not available on D2Q9");
        if (bc->product && bc->coupling != LBM_COUPLE_PASSIVE)
            return fail(nullptr, LBM_EUNSUPPORTED, "the product lattice needs PASSIVE coupling");
    } else if (bc->product && (bc->wall_diffuse != 0.0 || bc->wall_accommodation != 0.0))
        return fail(nullptr, LBM_EUNSUPPORTED, "the product lattice is not available with a diffuse wall");
    if (bc->product && bc->sputter == LBM_SPUTTER_STOCHASTIC)
        return fail(nullptr, LBM_EUNSUPPORTED, "the product lattice is not available with STOCHASTIC sputtering");
    if (bc->coupling < 0 || bc->coupling > 1) return fail(nullptr, LBM_EUNSUPPORTED, "unknown coupling mode");
    if (bc->species_x < 0 || bc->species_x > 2) return fail(nullptr, LBM_EUNSUPPORTED, "unknown species x-boundary");
    if (bc->storage < 0 || bc->storage > 3) return fail(nullptr, LBM_EUNSUPPORTED, "unknown storage format");
    if (!(bc->p_stick >= 0.0 && bc->p_stick <= 1.0)) return fail(nullptr, LBM_EINVAL, "p_stick must be in [0, 1]");
    if (!(bc->c_inlet >= 0.0) || !std::isfinite(bc->c_inlet)) return fail(nullptr, LBM_EINVAL, "c_inlet must be >= 0");
    if (!(bc->c0 >= 0.0) || !std::isfinite(bc->c0)) return fail(nullptr, LBM_EINVAL, "c0 must be >= 0");
    if (!(bc->rho0 > 0.0) || !std::isfinite(bc->rho0)) return fail(nullptr, LBM_EINVAL, "rho0 must be > 0");
    if (!std::isfinite(bc->c_ref)) return fail(nullptr, LBM_EINVAL, "c_ref must be finite");
    if (!(std::fabs(bc->store_ux) < 0.2)) return fail(nullptr, LBM_EINVAL, "store_ux must satisfy |store_ux| < 0.2");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(bc->force[a])) return fail(nullptr, LBM_EINVAL, "force must be finite");
    if (!(kn >= 0.0) || !std::isfinite(kn)) return fail(nullptr, LBM_EINVAL, "kn must be finite and >= 0");
    if (!(da > 0.0)) return fail(nullptr, LBM_EINVAL, "da must be > 0 (+inf allowed)");
    for (int k = 0; k < 2; ++k)
        if (!(tau[k] == 0.0 || tau[k] > 0.5) || !std::isfinite(tau[k]))
            return fail(nullptr, LBM_EINVAL, "tau must be 0 (derive) or > 1/2");
    if (tau[0] == 0.0 && kn == 0.0) return fail(nullptr, LBM_EINVAL, "give tau[0] or kn");
    const size_t n = size_t(g->nx) * g->ny * g->nz;
    for (size_t i = 0; i < n; ++i)
        if (g->voxels[i] > 2) return fail(nullptr, LBM_EINVAL, "voxel value > 2 at index " + std::to_string(i));
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_create(const lbm_geometry *g, double kn, double da, const double tau[2], const lbm_bc *bc,
                      lbm_ctx **out) {
    return lbm_create_on(g, kn, da, tau, bc, nullptr, out);
}

}  // extern "C"

namespace {

// Parameter maps: Eq. (knudsen) and Eq. (Da_def) with tau_ch = 1/p and
// tau_tr = delta / cs.
// ------------------------------------------------------------- D2Q9 path --
// Active links of the catalytic nodes of a plane (bit j: the source k - c_j
// is a gas node in the domain; x wraps only for a periodic species
// boundary), and the counts lbm_info reports.
struct Plane2D {
    std::vector<uint16_t> mask;
    int64_t nfluid = 0, niface = 0, nlinks = 0;
};

Plane2D plane_links(const uint8_t *vox, int nx, int ny, bool xper) {
    Plane2D p;
    p.mask.assign(size_t(nx) * ny, 0);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t k = size_t(y) * nx + x;
            if (vox[k] == LBM_FLUID) ++p.nfluid;
            if (vox[k] != LBM_CATALYTIC) continue;
            uint16_t m = 0;
            for (int j = 1; j < lbm2d::Q; ++j) {
                int sx = x - lbm2d::CX[j];
                const int sy = (y - lbm2d::CY[j] + ny) % ny;
                if (xper) sx = (sx + nx) % nx;
                if (sx < 0 || sx >= nx) continue;
                if (vox[size_t(sy) * nx + sx] == LBM_FLUID) m |= uint16_t(1u << j);
            }
            p.mask[k] = m;
            if (m) {
                ++p.niface;
                p.nlinks += __builtin_popcount(m);
            }
        }
    return p;
}

// Device bytes of a D2Q9 context: voxels, link masks, three arrays of Q
// populations per lattice (pre- and post-collision, emission), the running
// In sums, the partial sums and the totals.
int64_t plane_bytes(int64_t n, bool product) {
    const int64_t nb = lbm2d::blocks(n);
    const int64_t lat = product ? 3 : 2;
    return n + 2 * n + lat * 3 * lbm2d::Q * n * 8 + (lat - 1) * n * 8 + nb * (lbm2d::NPI + lbm2d::NPS) * 8 +
           lbm2d::NTOT * 8;
}

lbm_status create_plane(lbm_ctx *c, const lbm_geometry *g) {
    const int64_t n = c->n;
    Plane2D pl;
    try {
        pl = plane_links(g->voxels, g->nx, g->ny, c->ph.species_x == XB_PERIODIC);
        c->vox.assign(g->voxels, g->voxels + n);
    } catch (const std::bad_alloc &) {
        return fail(c, LBM_ENOMEM, "host allocation failed");
    }
    c->nfluid = pl.nfluid;
    c->niface = pl.niface;
    c->nlinks = pl.nlinks;
    lbm2d::Dev &d = c->d2;
    d.nx = g->nx;
    d.ny = g->ny;
    d.n = n;
    const bool prod = c->ph.product != 0;
    const size_t pop = size_t(lbm2d::Q) * size_t(n) * 8, nb = size_t(lbm2d::blocks(n));
    auto dbl = [&](size_t bytes) { return static_cast<double *>(dev_alloc(c, bytes)); };
    uint8_t *vox = static_cast<uint8_t *>(dev_alloc(c, size_t(n)));
    uint16_t *mask = static_cast<uint16_t *>(dev_alloc(c, size_t(n) * 2));
    d.vox = vox;
    d.mask = mask;
    d.fC = dbl(pop);
    d.fR = dbl(pop);
    d.pC = dbl(pop);
    d.pR = dbl(pop);
    d.em = dbl(pop);
    d.acc = dbl(size_t(n) * 8);
    if (prod) {
        d.fP = dbl(pop);
        d.pP = dbl(pop);
        d.emP = dbl(pop);
        d.accP = dbl(size_t(n) * 8);
    }
    d.part_i = dbl(nb * lbm2d::NPI * 8);
    d.part_s = dbl(nb * lbm2d::NPS * 8);
    d.tot = dbl(lbm2d::NTOT * 8);
    if (!vox || !mask || !d.fC || !d.fR || !d.pC || !d.pR || !d.em || !d.acc || !d.part_i || !d.part_s || !d.tot ||
        (prod && (!d.fP || !d.pP || !d.emP || !d.accP)))
        return fail(c, LBM_ENOMEM, "device allocation failed");
    lbm2d::Params &P = d.ph;
    P.tau_gas = c->ph.tau_gas;
    P.tau_species = c->ph.tau_species;
    P.p = c->ph.p;
    P.p_stick = c->ph.p_stick;
    P.p_stick_product = c->ph.p_stick_product;
    P.c_inlet = c->ph.c_inlet;
    P.force[0] = c->ph.force[0];
    P.force[1] = c->ph.force[1];
    P.sigma = c->ph.wall_diffuse;
    P.sputter = c->ph.sputter;
    P.coupling = c->ph.coupling;
    P.species_x = c->ph.species_x;
    P.product = c->ph.product;
    hipError_t e = hipMemcpyAsync(vox, g->voxels, size_t(n), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(mask, pl.mask.data(), size_t(n) * 2, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(d.tot, 0, lbm2d::NTOT * 8, c->stream);
    if (e == hipSuccess) e = lbm2d::launch_init(d, c->ph.rho0, c->ph.c0, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "D2Q9 set-up");
    return LBM_OK;
}

lbm_status plane_unsupported(lbm_ctx *c, const char *what) {
    return fail(c, LBM_EUNSUPPORTED, std::string(what) + " is not available on a D2Q9 context");
}

lbm_status step_plane(lbm_ctx *c, int64_t n) {
    for (int64_t k = 0; k < n; ++k) {
        const hipError_t e = lbm2d::launch_step(c->d2, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "D2Q9 step launch");
        c->step += 1;
    }
    return LBM_OK;
}

// Moments on the device into scratch buffers, copied to the host arrays
// (any may be NULL); with phi also rho_P and Phi_P.
lbm_status fields_plane(lbm_ctx *c, double *rho, double *u, double *conc, double *rhoP, double *phi) {
    const size_t n = size_t(c->n);
    double *buf = static_cast<double *>(scratch_alloc(c, (6 * n + size_t(c->nx)) * 8));
    if (!buf) return fail(c, LBM_ENOMEM, "field scratch allocation failed");
    double *d_rho = buf, *d_u = buf + n, *d_conc = buf + 4 * n, *d_rp = buf + 5 * n, *d_phi = buf + 6 * n;
    hipError_t e = lbm2d::launch_fields(c->d2, d_rho, d_u, d_conc, d_rp, phi ? d_phi : nullptr, c->stream);
    if (e == hipSuccess && rho) e = hipMemcpyAsync(rho, d_rho, n * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && u) e = hipMemcpyAsync(u, d_u, 3 * n * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && conc) e = hipMemcpyAsync(conc, d_conc, n * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && rhoP) e = hipMemcpyAsync(rhoP, d_rp, n * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && phi) e = hipMemcpyAsync(phi, d_phi, size_t(c->nx) * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    scratch_free(c, buf);
    if (e != hipSuccess) return hip_fail(c, e, "D2Q9 fields");
    return LBM_OK;
}

// Per node: factor times the running In sum at catalytic nodes, 0 elsewhere.
lbm_status plane_map(lbm_ctx *c, const double *d_acc, double factor, double *out) {
    std::vector<double> acc(size_t(c->n));
    hipError_t e = hipMemcpyAsync(acc.data(), d_acc, acc.size() * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "D2Q9 map copy");
    for (size_t k = 0; k < acc.size(); ++k) out[k] = c->vox[k] == LBM_CATALYTIC ? factor * acc[k] : 0.0;
    return LBM_OK;
}

lbm_status totals_plane(lbm_ctx *c, lbm_totals_t *t) {
    double v[lbm2d::NTOT];
    hipError_t e = hipMemcpyAsync(v, c->d2.tot, sizeof(v), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "D2Q9 totals copy");
    *t = lbm_totals_t{};
    t->step = c->step;
    t->mass_gas = v[0];
    t->mass_species = v[1];
    t->converted = v[2];
    t->lost = v[3];
    t->influx = v[4];
    t->outflux = v[5];
    t->mass_product = v[6];
    t->lost_product = v[7];
    t->product_out_inlet = v[8];
    t->product_out_outlet = v[9];
    t->nonfinite = v[10] != 0.0;
    if (t->nonfinite) return fail(c, LBM_ENONFINITE, "a global total became non-finite");
    return LBM_OK;
}

struct ParamMap {
    double tau_gas, tau_species, kn, p;
    int clamped;
    double wall_sigma;  // diffuse fraction of the gas wall in use
    int wall_clamped;   // 1 when the Kn relation had to clamp it to [0, 1]
};

// Diffuse fraction of the gas wall for Maxwell's first-order slip (J. C.
// Maxwell, Phil. Trans. R. Soc. 170, 231, 1879): slip length
// ((2 - sigma_v) / sigma_v) lambda with lambda = Kn delta (Eq. (knudsen)),
// sigma_v the tangential momentum accommodation.  The lattice wall (sigma
// diffuse, 1 - sigma bounced back) has, in force-driven flow between two
// planes delta nodes apart, the exact slip length
//   sigma (2 tau - 1) / (2 (2 - sigma)) + (16 tau^2 - 16 tau + 1) / (12 delta)
// (the second term is halfway bounce-back's, zero at (tau - 1/2)^2 = 3/16),
// so sigma / (2 - sigma) follows in closed form.  Clamped to [0, 1]: where
// the bounce-back slip of large tau already exceeds Maxwell's, sigma = 0.
double wall_sigma_for_slip(double tau, double delta, double accommodation, int *clamped) {
    const double maxwell = (2.0 - accommodation) / accommodation * (CS * (tau - 0.5) / delta) * delta;
    const double bounce = (16.0 * tau * tau - 16.0 * tau + 1.0) / (12.0 * delta);
    const double ratio = 2.0 * (maxwell - bounce) / (2.0 * tau - 1.0);  // sigma / (2 - sigma)
    *clamped = 0;
    if (!(ratio >= 0.0)) {
        *clamped = 1;
        return 0.0;
    }
    const double sigma = 2.0 * ratio / (1.0 + ratio);
    if (sigma > 1.0) {
        *clamped = 1;
        return 1.0;
    }
    return sigma;
}

lbm_status param_map(const lbm_geometry *g, double kn, double da, const double tau[2], const lbm_bc *bc,
                     ParamMap *m) {
    const double delta = g->pore_size;
    double tau_gas = tau[0];
    if (tau_gas == 0.0) tau_gas = 0.5 + kn * delta / CS;
    const double kn_of_tau = CS * (tau_gas - 0.5) / delta;
    if (tau[0] != 0.0 && kn != 0.0 && std::fabs(kn - kn_of_tau) > 1e-9 * std::max(1.0, kn))
        return fail(nullptr, LBM_EINVAL, "kn and tau[0] disagree");
    if (!(tau_gas > 0.5)) return fail(nullptr, LBM_EINVAL, "derived tau_gas must be > 1/2");
    m->tau_gas = tau_gas;
    m->tau_species = tau[1] != 0.0 ? tau[1] : tau_gas;
    m->kn = kn_of_tau;
    double p = std::isinf(da) ? 0.0 : CS / (da * delta);
    m->clamped = p > 1.0;
    m->p = m->clamped ? 1.0 : p;
    m->wall_sigma = bc->wall_diffuse;
    m->wall_clamped = 0;
    if (bc->wall_accommodation > 0.0)
        m->wall_sigma = wall_sigma_for_slip(tau_gas, delta, bc->wall_accommodation, &m->wall_clamped);
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_inspect(const lbm_geometry *g, double kn, double da, const double tau[2], const lbm_bc *bc,
                       lbm_info *info) {
    lbm_ctx *unused = nullptr;
    lbm_status st = validate(g, kn, da, tau, bc, &unused);
    if (st != LBM_OK) return st;
    if (!info) return fail(nullptr, LBM_EINVAL, "info is NULL");
    ParamMap m;
    st = param_map(g, kn, da, tau, bc, &m);
    if (st != LBM_OK) return st;
    if (bc->lattice == LBM_LATTICE_D2Q9) {
        try {
            const Plane2D pl = plane_links(g->voxels, g->nx, g->ny, bc->species_x == LBM_XBC_PERIODIC);
            *info = lbm_info{};
            info->tau_gas = m.tau_gas;
            info->tau_species = m.tau_species;
            info->kn = m.kn;
            info->p = m.p;
            info->da = da;
            info->pore_size = g->pore_size;
            info->p_clamped = m.clamped;
            info->wall_sigma = m.wall_sigma;
            info->wall_clamped = m.wall_clamped;
            info->storage = bc->storage;
            info->n_nodes = int64_t(g->nx) * g->ny;
            info->n_fluid = pl.nfluid;
            info->n_interface = pl.niface;
            info->n_catalytic_links = pl.nlinks;
            info->device_bytes = plane_bytes(info->n_nodes, bc->product != 0);
        } catch (const std::bad_alloc &) {
            return fail(nullptr, LBM_ENOMEM, "host allocation failed");
        }
        return LBM_OK;
    }
    try {
        lbm_ctx c;
        c.nx = g->nx;
        c.ny = g->ny;
        c.nz = g->nz;
        c.W = (g->nx + 63) / 64;
        c.n = int64_t(g->nx) * g->ny * g->nz;
        c.ph.species_x = bc->species_x;
        c.ph.sputter = bc->sputter;
        c.vox.assign(g->voxels, g->voxels + c.n);
        for (uint8_t v : c.vox) c.nfluid += v == LBM_FLUID;
        std::vector<uint32_t> ivox, imask;
        std::vector<double> iscale;
        build_interface(&c, ivox, imask, iscale);
        const int64_t nfp = (c.nfluid + 1 + 127) / 128 * 128;
        const int64_t sb = storage_bytes(bc->storage);
        const int64_t niface = int64_t(ivox.size());
        const int64_t rows = int64_t(g->ny) * g->nz;
        info->tau_gas = m.tau_gas;
        info->tau_species = m.tau_species;
        info->kn = m.kn;
        info->p = m.p;
        info->da = da;
        info->pore_size = g->pore_size;
        info->p_clamped = m.clamped;
        info->wall_sigma = m.wall_sigma;
        info->wall_clamped = m.wall_clamped;
        info->storage = bc->storage;
        info->n_nodes = c.n;
        info->n_fluid = c.nfluid;
        info->n_interface = niface;
        info->n_catalytic_links = c.nlinks;
        // the buffers lbm_create allocates (populations and emission, chunk
        // records and traversal tables, interface arrays, coordinates, wave
        // order and wave units of the compact sweep, partial sums), each
        // rounded up to 256 B
        auto r256 = [](int64_t b) { return std::max<int64_t>((b + 255) / 256 * 256, 256); };
        const int64_t chunks = rows * c.W;
        const bool compact = g->ny <= 1024 && g->nz <= 1024 && c.nfluid > 0;
        // partial-sum rows: the larger of the chunk sweep's blocks (four
        // wavefronts each) and the compact sweep's (one wavefront each)
        const int64_t blocks = std::max(((chunks + 3) / 4 + 7) / 8 * 8, compact ? ((c.nfluid + 63) / 64 + 7) / 8 * 8 : 0);
        const int64_t ns = bc->sputter == LBM_SPUTTER_STOCHASTIC ? NSLOT : 1;
        int64_t bytes = r256((76 * nfp + ns * niface + 1) * sb) + r256(chunks * int64_t(sizeof(ChunkInfo))) +
                        r256(chunks * 4) + 2 * r256(niface * 4) + 2 * r256(niface * 8) + r256(ns * niface * 8) +
                        r256((4 * blocks + 2 * ((niface + 255) / 256) + 2 * FOLD_BLOCKS * NPART) * 8) +
                        r256(int64_t(sizeof(DevTotals)));
        if (compact) bytes += r256(nfp * 4) + 2 * r256((c.nfluid + 63) / 64 * 4);
        if (bc->product) {
            // P buffers and E_P, In_P and Acc_P, P partial sums
            const int64_t rows_p = blocks;  // as for the sweep partials above
            bytes += r256((38 * nfp + niface + 1) * sb) + 2 * r256(niface * 8) +
                     r256((3 * rows_p + 2 * ((niface + 255) / 256)) * 8);
        }
        info->device_bytes = bytes;
    } catch (const std::bad_alloc &) {
        return fail(nullptr, LBM_ENOMEM, "host allocation failed");
    }
    return LBM_OK;
}

lbm_status lbm_create_on(const lbm_geometry *g, double kn, double da, const double tau[2], const lbm_bc *bc,
                         const lbm_device *dev, lbm_ctx **out) {
    lbm_status st = validate(g, kn, da, tau, bc, out);
    if (st != LBM_OK) return st;
    ParamMap m;
    st = param_map(g, kn, da, tau, bc, &m);
    if (st != LBM_OK) return st;
    const double delta = g->pore_size;
    const double tau_gas = m.tau_gas, tau_species = m.tau_species, kn_of_tau = m.kn, p = m.p;
    const int clamped = m.clamped;
    const double wall_sigma = m.wall_sigma;
    const int wall_clamped = m.wall_clamped;

    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return hip_fail(nullptr, e, "no HIP device");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, LBM_EDEVICE, std::string("this library is built for gfx950, device is ") + prop.gcnArchName);

    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(nullptr, LBM_ENOMEM, "host allocation failed");
    if (dev) c->dev = *dev;
    c->stream = static_cast<hipStream_t>(c->dev.stream);
    c->device = device;
    c->nx = g->nx;
    c->ny = g->ny;
    c->nz = g->nz;
    c->W = (g->nx + 63) / 64;
    c->n = int64_t(g->nx) * g->ny * g->nz;
    c->kn = kn_of_tau;
    c->da = da;
    c->delta = delta;
    c->p = p;
    c->p_clamped = clamped;
    c->wall_clamped = wall_clamped;
    c->ph.tau_gas = tau_gas;
    c->ph.tau_species = tau_species;
    for (int a = 0; a < 3; ++a) c->ph.force[a] = bc->force[a];
    c->ph.rho0 = bc->rho0;
    c->ph.c0 = bc->c0;
    c->ph.c_inlet = bc->species_x != LBM_XBC_PERIODIC ? bc->c_inlet : 0.0;
    c->ph.rho_ref = bc->rho0;
    // the reference flow of the carrier's shifted form (D3Q19; not with FP32
    // storage, whose sweep has no registers to spare for it)
    c->ph.store_ux = bc->lattice == LBM_LATTICE_D3Q19 && bc->storage != LBM_STORE_F32 ? bc->store_ux : 0.0;
    // Species populations are stored unshifted by default (c_ref = 0): the
    // concentration is depleted next to the catalyst, and a shift would cost
    // relative precision exactly where the conversion is decided.
    c->ph.c_ref = bc->c_ref >= 0.0 ? bc->c_ref : 0.0;
    // Fixed-point scale 2^S of the In(k) sums: reactant populations are of the
    // order of the largest of c_inlet, c0 and c_ref (c); with S = 47 -
    // ceil(log2 c) a term up to 16 c stays below the 2^51 the rounding allows,
    // and 18 such terms below 2^56 in the signed 64-bit sum.
    {
        const double c_scale = std::max(std::max(c->ph.c_inlet, bc->c0), std::max(c->ph.c_ref, 1e-300));
        const int shift = std::min(900, std::max(-900, 47 - int(std::ceil(std::log2(c_scale)))));
        c->ph.in_scale = std::ldexp(1.0, shift);
        c->ph.in_unscale = std::ldexp(1.0, -shift);
    }
    c->ph.p_stick = bc->p_stick;
    c->ph.p = p;
    c->ph.sputter = bc->sputter;
    c->ph.coupling = bc->coupling;
    c->ph.species_x = bc->species_x;
    c->ph.storage = bc->storage;
    c->ph.product = bc->product;
    c->ph.p_stick_product = bc->product ? bc->p_stick_product : 0.0;
    c->ph.seed = bc->seed;
    c->ph.wall_diffuse = wall_sigma;
    c->ph.rounding = bc->rounding;
    c->ph.step_ctr = 0;  // the initial state is the collision of step 0
    c->ph.emission_gather = 1;  // measured faster for a single context at 256^3 (LBM_TUNE_EMISSION)

    if (bc->lattice == LBM_LATTICE_D2Q9) {
        c->lattice = LBM_LATTICE_D2Q9;
        st = create_plane(c, g);
        if (st != LBM_OK) {
            g_create_error = c->err;
            lbm_destroy(c);
            return st;
        }
        *out = c;
        return LBM_OK;
    }

    try {
        c->vox.assign(g->voxels, g->voxels + c->n);
        c->geom_hash = fnv1a(c->vox.data(), c->vox.size());
        c->nfluid = 0;
        for (uint8_t v : c->vox) c->nfluid += v == LBM_FLUID;
        // one spare element per direction array at least: the last one holds
        // the inlet ghost population of the reactant
        c->nfp = (c->nfluid + 1 + 127) / 128 * 128;
        // Population layout: blocks of 64 consecutive nodes holding all 19
        // slots when a whole pair buffer fits the kernels' 32-bit offsets (a
        // wavefront then reads its own and its neighbours' populations from
        // few contiguous blocks and writes one), else slot-major.
        if (uint64_t(19) * uint64_t(c->nfp) * 2 * uint64_t(storage_bytes(bc->storage)) < (uint64_t(1) << 32)) {
            c->lay_ss = 64;
            c->lay_bs = 19 * 64;
        } else {
            c->lay_ss = uint32_t(c->nfp);
            c->lay_bs = 64;
        }
        std::vector<uint32_t> ivox, imask;
        std::vector<double> iscale;
        build_interface(c, ivox, imask, iscale);
        c->niface = int64_t(ivox.size());
        c->iface_vox = ivox;
        if (c->nfluid >= int64_t(NB_IDX) || c->niface >= int64_t(NB_IDX)) {
            release(c);
            delete c;
            return fail(nullptr, LBM_EUNSUPPORTED, "more than 2^30 gas or interface nodes");
        }
        std::vector<ChunkInfo> chunks;
        build_chunks(c, ivox, chunks);
        c->nwaves = (c->nfluid + 63) / 64;
        // node-compact sweep tables (coordinates packed as x | y << 12 | z << 22)
        c->compact_ok = c->ny <= 1024 && c->nz <= 1024 && c->nfluid > 0;
        std::vector<uint32_t> pos, worder, wunits;
        if (c->compact_ok) {
            pos.assign(size_t(c->nfp), 0);
            size_t r = 0;
            for (int z = 0; z < c->nz; ++z)
                for (int y = 0; y < c->ny; ++y)
                    for (int x = 0; x < c->nx; ++x)
                        if (c->vox[size_t((int64_t(z) * c->ny + y) * c->nx + x)] == LBM_FLUID)
                            pos[r++] = uint32_t(x) | (uint32_t(y) << 12) | (uint32_t(z) << 22);
            build_wave_order(c, pos, std::min(c->ytile, c->ny), worder);
            build_wave_units(c, pos, wunits);
            c->compact = 1;
        }
        if (c->ph.product && !c->compact_ok) {
            release(c);
            delete c;
            return fail(nullptr, LBM_EUNSUPPORTED, "the product lattice needs the node-compact sweep (ny, nz <= 1024)");
        }

        // The kernels address every buffer with 32-bit byte offsets from a
        // scalar base: two adjacent direction arrays (2 nfp elements of two
        // populations each) and the emission array (one population per
        // interface node) must each stay below 4 GiB.
        {
            const uint64_t sbytes = uint64_t(storage_bytes(c->ph.storage)), lim = uint64_t(1) << 32;
            if (4 * uint64_t(c->nfp) * sbytes >= lim || uint64_t(nslot(c) * c->niface) * sbytes >= lim ||
                uint64_t(nslot(c) * c->niface) >= (uint64_t(1) << 32)) {
                release(c);
                delete c;
                return fail(nullptr, LBM_EUNSUPPORTED,
                            "lattice too large for this storage type (a buffer would exceed 4 GiB of 32-bit offsets)");
            }
        }
        const Geometry gtmp = geometry(c);
        c->blocks_sweep = sweep_blocks(gtmp);
        c->part_rows = std::max(c->blocks_sweep, c->compact_ok ? sweep_blocks_c(gtmp) : int64_t(0));
        c->blocks_iface = interface_blocks(c->niface);

        const int sb = storage_bytes(c->ph.storage);
        c->d_chunks = static_cast<ChunkInfo *>(dev_alloc(c, chunks.size() * sizeof(ChunkInfo)));
        c->d_order = static_cast<uint32_t *>(dev_alloc(c, chunks.size() * sizeof(uint32_t)));
        std::vector<uint32_t> order(chunks.size());
        c->ytile = std::min(c->ytile, c->ny);
        build_order(c->nx, c->ny, c->nz, c->ytile, order.data());
        c->d_iface_vox = static_cast<uint32_t *>(dev_alloc(c, ivox.size() * 4));
        c->d_iface_mask = static_cast<uint32_t *>(dev_alloc(c, imask.size() * 4));
        c->d_iface_scale = static_cast<double *>(dev_alloc(c, iscale.size() * 8));
        c->d_acc = static_cast<double *>(dev_alloc(c, size_t(c->niface) * 8));
        c->d_inacc = static_cast<unsigned long long *>(dev_alloc(c, size_t(nslot(c) * c->niface) * 8));
        if (c->compact_ok) {
            c->d_pos = static_cast<uint32_t *>(dev_alloc(c, pos.size() * 4));
            c->d_worder = static_cast<uint32_t *>(dev_alloc(c, worder.size() * 4));
            c->d_wunits = static_cast<uint32_t *>(dev_alloc(c, wunits.size() * 4));
        }
        // One pool: population buffers A and B, then the emission array (one
        // element per interface node, indexed by interface index, plus one:
        // the sweeps load element 0 for lanes without a catalytic source,
        // which must exist when there is no interface node).
        char *pool = static_cast<char *>(dev_alloc(c, (size_t(76) * c->nfp + size_t(nslot(c) * c->niface) + 1) * sb));
        if (pool) {
            c->d_pop[0] = pool;
            c->d_pop[1] = pool + size_t(38) * c->nfp * sb;
            c->d_emit = pool + size_t(76) * c->nfp * sb;
        }
        const int64_t nparts = 4 * c->part_rows + 2 * c->blocks_iface + 2 * FOLD_BLOCKS * NPART;
        c->d_part = static_cast<double *>(dev_alloc(c, size_t(nparts) * 8));
        c->d_tot = static_cast<DevTotals *>(dev_alloc(c, sizeof(DevTotals)));
        bool prod_ok = true;
        if (c->ph.product) {
            // P buffers A and B, then E_P (one element per interface node)
            char *pp = static_cast<char *>(dev_alloc(c, (size_t(38) * c->nfp + size_t(c->niface) + 1) * sb));
            if (pp) {
                c->d_popP[0] = pp;
                c->d_popP[1] = pp + size_t(19) * c->nfp * sb;
                c->d_emitP = pp + size_t(38) * c->nfp * sb;
            }
            c->d_inaccP = static_cast<unsigned long long *>(dev_alloc(c, size_t(c->niface) * 8));
            c->d_accP = static_cast<double *>(dev_alloc(c, size_t(c->niface) * 8));
            c->rows_partP = std::max(c->blocks_sweep, sweep_blocks_c(gtmp));
            c->d_partP = static_cast<double *>(dev_alloc(c, size_t(3 * c->rows_partP + 2 * c->blocks_iface) * 8));
            prod_ok = pp && c->d_inaccP && c->d_accP && c->d_partP;
        }
        if (!c->d_chunks || !c->d_order || !c->d_inacc || !c->d_iface_vox || !c->d_iface_mask || !c->d_iface_scale || !c->d_acc || !c->d_emit ||
            !c->d_pop[0] || !c->d_pop[1] || !c->d_part || !c->d_tot || !prod_ok ||
            (c->compact_ok && (!c->d_pos || !c->d_worder || !c->d_wunits))) {
            release(c);
            delete c;
            return fail(nullptr, LBM_ENOMEM, "device allocation failed");
        }
        auto up = [&](void *d, const void *h, size_t bytes) {
            if (bytes && e == hipSuccess) e = hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, c->stream);
        };
        e = hipSuccess;
        up(c->d_chunks, chunks.data(), chunks.size() * sizeof(ChunkInfo));
        up(c->d_order, order.data(), order.size() * sizeof(uint32_t));
        up(c->d_iface_vox, ivox.data(), ivox.size() * 4);
        up(c->d_iface_mask, imask.data(), imask.size() * 4);
        up(c->d_iface_scale, iscale.data(), iscale.size() * 8);

        if (c->compact_ok) {
            up(c->d_pos, pos.data(), pos.size() * 4);
            up(c->d_worder, worder.data(), worder.size() * 4);
            up(c->d_wunits, wunits.data(), wunits.size() * 4);
        }
        if (e == hipSuccess) e = hipMemsetAsync(c->d_acc, 0, size_t(c->niface) * 8, c->stream);
        if (e == hipSuccess) e = hipMemsetAsync(c->d_emit, 0, (size_t(nslot(c) * c->niface) + 1) * sb, c->stream);
        DevTotals t0{};
        t0.mass_gas = double(c->nfluid) * bc->rho0;
        t0.mass_species = double(c->nfluid) * bc->c0;
        up(c->d_tot, &t0, sizeof(t0));
        if (e == hipSuccess) e = launch_init(geometry(c), c->ph, c->d_pop[1], c->d_pop[0], c->stream);
        if (e == hipSuccess) e = launch_in_init(geometry(c), c->ph, interface_list(c), c->d_pop[0], c->stream);
        if (c->ph.product) {
            // no product anywhere at the start: both P buffers, E_P and Acc_P are 0
            if (e == hipSuccess)
                e = hipMemsetAsync(c->d_popP[0], 0, (size_t(38) * c->nfp + size_t(c->niface) + 1) * sb, c->stream);
            if (e == hipSuccess && c->niface) e = hipMemsetAsync(c->d_accP, 0, size_t(c->niface) * 8, c->stream);
            if (e == hipSuccess)
                e = launch_in_init_product(geometry(c), c->ph, interface_list(c), c->d_popP[0], c->d_inaccP,
                                           c->stream);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);  // host vectors go out of scope
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&c->h_flag), sizeof(int32_t));
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->flag_event, hipEventDisableTiming);
        if (e != hipSuccess) {
            lbm_status s = hip_fail(nullptr, e, "create");
            release(c);
            delete c;
            return s;
        }
        *c->h_flag = 0;
        c->cur = 0;
    } catch (const std::bad_alloc &) {
        release(c);
        delete c;
        return fail(nullptr, LBM_ENOMEM, "host allocation failed");
    }
    *out = c;
    return LBM_OK;
}

lbm_status lbm_step(lbm_ctx *c, int64_t n) {
    if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
    if (n < 0) return fail(c, LBM_EINVAL, "n must be >= 0");
    if (c->lattice == LBM_LATTICE_D2Q9) return step_plane(c, n);
    lbm_status st = check_pending_flag(c);
    if (st != LBM_OK) return st;
    // the reductions of step s run in the front launches of steps s + 1 and
    // s + 2 of this call; the last step closes the call's own
    for (int64_t s = 0; s < n; ++s) {
        st = one_step(c, s >= 1, s >= 2, s == n - 1);
        if (st != LBM_OK) return st;
    }
    if (n > 0) {
        hipError_t e = hipMemcpyAsync(c->h_flag, &c->d_tot->nonfinite, sizeof(int32_t), hipMemcpyDeviceToHost,
                                      c->stream);
        if (e == hipSuccess) e = hipEventRecord(c->flag_event, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "watchdog copy");
        c->flag_pending = true;
    }
    return LBM_OK;
}

static lbm_status fields_impl(lbm_ctx *c, void *rho, void *u, void *conc, bool f64) {
    const int mode = c->step == 0 ? 2 : 1;
    const void *fin = c->d_pop[1 - c->cur];
    hipError_t e = launch_fields(geometry(c), c->ph, fin, c->d_emit, mode, rho, u, conc, f64, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "fields kernel launch");
    return LBM_OK;
}

lbm_status lbm_fields(lbm_ctx *c, double *rho, double *u, double *conc) {
    if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
    if (c->lattice == LBM_LATTICE_D2Q9) return fields_plane(c, rho, u, conc, nullptr, nullptr);
    const size_t n = size_t(c->n);
    double *d[3] = {nullptr, nullptr, nullptr};
    double *h[3] = {rho, u, conc};
    const size_t len[3] = {n, 3 * n, n};
    for (int k = 0; k < 3; ++k) {
        if (!h[k]) continue;
        void *p = nullptr;
        if (c->dev.alloc)
            p = c->dev.alloc(len[k] * 8, c->dev.user);
        else if (hipMalloc(&p, len[k] * 8) != hipSuccess)
            p = nullptr;
        if (!p) {
            for (int j = 0; j < k; ++j)
                if (d[j]) (c->dev.free ? c->dev.free(d[j], c->dev.user) : (void)hipFree(d[j]));
            return fail(c, LBM_ENOMEM, "fields scratch allocation failed");
        }
        d[k] = static_cast<double *>(p);
    }
    lbm_status st = fields_impl(c, d[0], d[1], d[2], true);
    hipError_t e = hipSuccess;
    for (int k = 0; k < 3 && st == LBM_OK; ++k)
        if (h[k] && e == hipSuccess) e = hipMemcpyAsync(h[k], d[k], len[k] * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    for (int k = 0; k < 3; ++k)
        if (d[k]) (c->dev.free ? c->dev.free(d[k], c->dev.user) : (void)hipFree(d[k]));
    if (st != LBM_OK) return st;
    if (e != hipSuccess) return hip_fail(c, e, "fields copy");
    return LBM_OK;
}

lbm_status lbm_fields_noalloc(lbm_ctx *c, double *rho, double *u, double *conc) {
    if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
    if (c->lattice == LBM_LATTICE_D2Q9) return plane_unsupported(c, "lbm_fields_noalloc");
    if (!rho && !u && !conc) return LBM_OK;
    // whole x-rows per pass through the device scratch: rho, three velocity
    // components and conc, 5 nx doubles a row
    const int64_t rows = int64_t(c->ny) * c->nz, n = c->n;
    const int64_t per_pass = FIELDS_SCRATCH_DOUBLES / (5 * int64_t(c->nx));
    if (per_pass < 1) return fail(c, LBM_EINVAL, "one x-row of fields exceeds the 32 MiB scratch");
    int prev = -1;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return hip_fail(c, e, "hipGetDevice");
    if (prev != c->device) {
        e = hipSetDevice(c->device);
        if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    }
    double *scr = nullptr;
    e = scratch_address(c->device, &scr);
    if (e == hipSuccess) {
        const int mode = c->step == 0 ? 2 : 1;
        const void *fin = c->d_pop[1 - c->cur];
        const Geometry g = geometry(c);
        for (int64_t r0 = 0; r0 < rows && e == hipSuccess; r0 += per_pass) {
            const int64_t r1 = std::min(rows, r0 + per_pass);
            const int64_t len = (r1 - r0) * c->nx, off = r0 * c->nx;
            double *s_rho = scr, *s_u = scr + len, *s_c = scr + 4 * len;
            e = launch_fields_rows(g, c->ph, fin, c->d_emit, mode, rho ? s_rho : nullptr, u ? s_u : nullptr,
                                   conc ? s_c : nullptr, true, r0, r1, len, c->stream);
            // the next pass's kernel is queued behind these copies on the same stream
            if (e == hipSuccess && rho)
                e = hipMemcpyAsync(rho + off, s_rho, size_t(len) * 8, hipMemcpyDeviceToHost, c->stream);
            for (int a = 0; a < 3 && e == hipSuccess && u; ++a)
                e = hipMemcpyAsync(u + a * n + off, s_u + a * len, size_t(len) * 8, hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess && conc)
                e = hipMemcpyAsync(conc + off, s_c, size_t(len) * 8, hipMemcpyDeviceToHost, c->stream);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    if (prev != c->device) (void)hipSetDevice(prev);
    if (e != hipSuccess) return hip_fail(c, e, "allocation-free fields");
    return LBM_OK;
}

lbm_status lbm_stream_copy(void *dst, const void *src, size_t bytes, void *stream) {
    if (!dst || !src) return fail(nullptr, LBM_EINVAL, "NULL argument");
    if (bytes % 16 != 0 || (reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16 != 0)
        return fail(nullptr, LBM_EINVAL, "bytes and both pointers must be multiples of 16");
    const hipError_t e = launch_stream_copy(dst, src, bytes, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(nullptr, e, "stream copy launch");
    return LBM_OK;
}

lbm_status lbm_stream_pull(void *dst, const void *src, int32_t nx, int32_t ny, int32_t nz, int32_t pair_bytes,
                           void *stream) {
    if (!dst || !src) return fail(nullptr, LBM_EINVAL, "NULL argument");
    if (nx < 1 || ny < 1 || nz < 1 || ny > 65535 || nz > 65535)
        return fail(nullptr, LBM_EINVAL, "nx, ny, nz must be >= 1, ny and nz <= 65535");
    if (uint64_t(nx) * uint64_t(ny) * uint64_t(nz) > (uint64_t(1) << 27))  // element indices stay 32-bit
        return fail(nullptr, LBM_EINVAL, "nx ny nz must not exceed 2^27 nodes");
    if (pair_bytes != 4 && pair_bytes != 8 && pair_bytes != 16)
        return fail(nullptr, LBM_EINVAL, "pair_bytes must be 4, 8 or 16");
    const uintptr_t a = reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src);
    if (a % uintptr_t(pair_bytes) != 0) return fail(nullptr, LBM_EINVAL, "pointers must be aligned to pair_bytes");
    const uint64_t bytes = stream_pull_elements(nx, ny, nz) * uint64_t(pair_bytes);
    const uintptr_t d = reinterpret_cast<uintptr_t>(dst), r = reinterpret_cast<uintptr_t>(src);
    if (d < r + bytes && r < d + bytes) return fail(nullptr, LBM_EINVAL, "the buffers must not overlap");
    const hipError_t e = launch_stream_pull(dst, src, nx, ny, nz, pair_bytes, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(nullptr, e, "stream pull launch");
    return LBM_OK;
}

lbm_status lbm_fields_device(lbm_ctx *c, float *rho, float *u, float *conc) {
    if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
    if (c->lattice == LBM_LATTICE_D2Q9) return plane_unsupported(c, "lbm_fields_device");
    return fields_impl(c, rho, u, conc, false);
}

lbm_status lbm_populations(lbm_ctx *c, const int32_t origin[3], const int32_t extent[3], double *fC, double *fR) {
    if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
    if (c->lattice == LBM_LATTICE_D2Q9) return plane_unsupported(c, "lbm_populations");
    if (!origin || !extent || !fC || !fR) return fail(c, LBM_EINVAL, "NULL argument");
    const int dims[3] = {c->nx, c->ny, c->nz};
    for (int a = 0; a < 3; ++a)
        if (origin[a] < 0 || extent[a] < 1 || int64_t(origin[a]) + extent[a] > dims[a])
            return fail(c, LBM_EINVAL, "box must lie inside the lattice with extent >= 1");
    const Window win{origin[0], origin[1], origin[2], extent[0], extent[1], extent[2]};
    const size_t len = size_t(19) * size_t(extent[0]) * size_t(extent[1]) * size_t(extent[2]);
    double *d[2] = {nullptr, nullptr};
    for (int k = 0; k < 2; ++k) {
        void *p = nullptr;
        if (c->dev.alloc)
            p = c->dev.alloc(len * 8, c->dev.user);
        else if (hipMalloc(&p, len * 8) != hipSuccess)
            p = nullptr;
        if (!p) {
            if (d[0]) (c->dev.free ? c->dev.free(d[0], c->dev.user) : (void)hipFree(d[0]));
            return fail(c, LBM_ENOMEM, "populations scratch allocation failed");
        }
        d[k] = static_cast<double *>(p);
    }
    hipError_t e = hipMemsetAsync(d[0], 0, len * 8, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(d[1], 0, len * 8, c->stream);
    if (e == hipSuccess)
        e = launch_populations(geometry(c), c->ph, c->d_pop[1 - c->cur], c->d_emit, c->step == 0 ? 2 : 1, win, d[0],
                               d[1], c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(fC, d[0], len * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(fR, d[1], len * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    for (int k = 0; k < 2; ++k) (c->dev.free ? c->dev.free(d[k], c->dev.user) : (void)hipFree(d[k]));
    if (e != hipSuccess) return hip_fail(c, e, "populations");
    return LBM_OK;
}

lbm_status lbm_conversion_map(lbm_ctx *c, double *conv) {
    if (!c || !conv) return fail(c, LBM_EINVAL, "NULL argument");
    if (c->lattice == LBM_LATTICE_D2Q9) return plane_map(c, c->d2.acc, c->ph.p * c->ph.p_stick, conv);
    std::vector<double> acc(size_t(c->niface));
    hipError_t e = hipSuccess;
    if (c->niface) e = hipMemcpyAsync(acc.data(), c->d_acc, acc.size() * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "conversion map copy");
    std::memset(conv, 0, size_t(c->n) * sizeof(double));
    const double f = c->ph.p * c->ph.p_stick;
    for (size_t k = 0; k < acc.size(); ++k) conv[c->iface_vox[k]] = f * acc[k];
    return LBM_OK;
}

lbm_status lbm_product_fields(lbm_ctx *c, double *conc, double *stuck, double *phi) {
    if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
    if (!c->ph.product) return fail(c, LBM_EUNSUPPORTED, "this context has no product lattice");
    if (c->lattice == LBM_LATTICE_D2Q9) {
        if (stuck) {
            const lbm_status st = plane_map(c, c->d2.accP, c->ph.p_stick_product, stuck);
            if (st != LBM_OK) return st;
        }
        return conc || phi ? fields_plane(c, nullptr, nullptr, nullptr, conc, phi) : LBM_OK;
    }
    hipError_t e = hipSuccess;
    if (stuck) {
        std::vector<double> acc(size_t(c->niface));
        if (c->niface) e = hipMemcpyAsync(acc.data(), c->d_accP, acc.size() * 8, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "product map copy");
        std::memset(stuck, 0, size_t(c->n) * sizeof(double));
        for (size_t k = 0; k < acc.size(); ++k) stuck[c->iface_vox[k]] = c->ph.p_stick_product * acc[k];
    }
    if (!conc && !phi) return LBM_OK;
    // device temporaries: rho_P, and for phi the carrier velocity
    const size_t n = size_t(c->n);
    double *d_c = static_cast<double *>(scratch_alloc(c, n * 8));
    double *d_u = phi ? static_cast<double *>(scratch_alloc(c, 3 * n * 8)) : nullptr;
    double *d_phi = phi ? static_cast<double *>(scratch_alloc(c, size_t(c->nx) * 8)) : nullptr;
    if (!d_c || (phi && (!d_u || !d_phi))) {
        scratch_free(c, d_c);
        scratch_free(c, d_u);
        scratch_free(c, d_phi);
        return fail(c, LBM_ENOMEM, "product field scratch allocation failed");
    }
    const int mode = c->step == 0 ? 2 : 1;
    const Geometry g = geometry(c);
    // the buffers the last sweep pulled from (at step 0 the stored initial
    // state), as for lbm_fields
    const void *fin = c->d_pop[1 - c->cur];
    const void *finp = c->d_popP[1 - c->cur];
    e = launch_product_field(g, c->ph, fin, finp, c->d_emitP, mode, d_c, c->stream);
    if (e == hipSuccess && phi) e = launch_fields(g, c->ph, fin, c->d_emit, mode, nullptr, d_u, nullptr, true, c->stream);
    if (e == hipSuccess && phi) e = launch_flux_profile(g, d_c, d_u, d_phi, c->stream);
    if (e == hipSuccess && conc) e = hipMemcpyAsync(conc, d_c, n * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && phi) e = hipMemcpyAsync(phi, d_phi, size_t(c->nx) * 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    scratch_free(c, d_c);
    scratch_free(c, d_u);
    scratch_free(c, d_phi);
    if (e != hipSuccess) return hip_fail(c, e, "product fields");
    return LBM_OK;
}

lbm_status lbm_totals(lbm_ctx *c, lbm_totals_t *t) {
    if (!c || !t) return fail(c, LBM_EINVAL, "NULL argument");
    if (c->lattice == LBM_LATTICE_D2Q9) return totals_plane(c, t);
    DevTotals d;
    hipError_t e = hipMemcpyAsync(&d, c->d_tot, sizeof(d), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "totals copy");
    t->step = c->step;
    t->mass_gas = d.mass_gas;
    t->mass_species = d.mass_species;
    t->converted = d.converted;
    t->lost = d.lost;
    t->influx = d.influx;
    t->outflux = d.outflux;
    t->nonfinite = d.nonfinite;
    t->reserved = 0;
    t->mass_product = d.mass_product;
    t->lost_product = d.lost_product;
    t->product_out_inlet = d.product_out_inlet;
    t->product_out_outlet = d.product_out_outlet;
    if (d.nonfinite) return fail(c, LBM_ENONFINITE, "a global total became non-finite");
    return LBM_OK;
}

lbm_status lbm_query(const lbm_ctx *c, lbm_info *info) {
    if (!c || !info) return LBM_EINVAL;
    info->tau_gas = c->ph.tau_gas;
    info->tau_species = c->ph.tau_species;
    info->kn = c->kn;
    info->p = c->p;
    info->da = c->da;
    info->pore_size = c->delta;
    info->p_clamped = c->p_clamped;
    info->wall_sigma = c->ph.wall_diffuse;
    info->wall_clamped = c->wall_clamped;
    info->storage = c->ph.storage;
    info->n_nodes = c->n;
    info->n_fluid = c->nfluid;
    info->n_interface = c->niface;
    info->n_catalytic_links = c->nlinks;
    info->device_bytes = c->device_bytes;
    return LBM_OK;
}

lbm_status lbm_active_links(const lbm_ctx *c, uint8_t *b) {
    if (!c || !b) return LBM_EINVAL;
    if (c->lattice == LBM_LATTICE_D2Q9) {
        const Plane2D pl = plane_links(c->vox.data(), c->nx, c->ny, c->ph.species_x == XB_PERIODIC);
        for (size_t k = 0; k < pl.mask.size(); ++k) b[k] = uint8_t(__builtin_popcount(pl.mask[k]));
        return LBM_OK;
    }
    std::memset(b, 0, size_t(c->n));
    const bool xper = c->ph.species_x == XB_PERIODIC;
    // recount from the voxel map, the same rule the interface list uses
    for (int z = 0; z < c->nz; ++z)
        for (int y = 0; y < c->ny; ++y)
            for (int x = 0; x < c->nx; ++x) {
                const int64_t k = (int64_t(z) * c->ny + y) * c->nx + x;
                if (c->vox[size_t(k)] != LBM_CATALYTIC) continue;
                int cnt = 0;
                for (int j = 1; j < 19; ++j) {
                    int xs = x - CX[j];
                    const int ys = (y - CY[j] + c->ny) % c->ny, zs = (z - CZ[j] + c->nz) % c->nz;
                    if (xs < 0 || xs >= c->nx) {
                        if (!xper) continue;
                        xs = (xs + c->nx) % c->nx;
                    }
                    cnt += c->vox[size_t((int64_t(zs) * c->ny + ys) * c->nx + xs)] == LBM_FLUID;
                }
                b[k] = uint8_t(cnt);
            }
    return LBM_OK;
}

lbm_status lbm_synchronize(lbm_ctx *c) {
    if (!c) return LBM_EINVAL;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "synchronize");
    return check_pending_flag(c);
}

lbm_status lbm_set_tunable(lbm_ctx *c, int32_t which, int64_t value) {
    if (!c) return LBM_EINVAL;
    if (c->lattice == LBM_LATTICE_D2Q9) return plane_unsupported(c, "lbm_set_tunable");
    if (which == LBM_TUNE_YTILE) {
        if (value < 1 || value > c->ny) return fail(c, LBM_EINVAL, "ytile must be in [1, ny]");
        if (int(value) == c->ytile) return LBM_OK;
        std::vector<uint32_t> order(size_t(int64_t(c->ny) * c->nz * c->W));
        build_order(c->nx, c->ny, c->nz, int(value), order.data());
        // the stream may still be reading the old table
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess)
            e = hipMemcpy(c->d_order, order.data(), order.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(c, e, "traversal table upload");
        if (c->compact_ok) {
            std::vector<uint32_t> pos(size_t(c->nwaves) * 64), worder;
            e = hipMemcpy(pos.data(), c->d_pos, std::min(pos.size(), size_t(c->nfp)) * 4, hipMemcpyDeviceToHost);
            if (e == hipSuccess) {
                build_wave_order(c, pos, int(value), worder);
                e = hipMemcpy(c->d_worder, worder.data(), worder.size() * 4, hipMemcpyHostToDevice);
            }
            if (e != hipSuccess) return hip_fail(c, e, "wave order upload");
        }
        c->ytile = int(value);
        return LBM_OK;
    }
    if (which == LBM_TUNE_SWEEP) {
        if (value != 0 && value != 1) return fail(c, LBM_EINVAL, "sweep variant must be 0 or 1");
        if (value == 1 && !c->compact_ok)
            return fail(c, LBM_EUNSUPPORTED, "the node-compact sweep needs ny, nz <= 1024 and a gas node");
        if (value == 0 && c->ph.product)
            return fail(c, LBM_EUNSUPPORTED, "the product lattice runs on the node-compact sweep only");
        c->compact = int(value);
        return LBM_OK;
    }
    if (which == LBM_TUNE_EMISSION) {
        if (value != 0 && value != 1) return fail(c, LBM_EINVAL, "emission read mode must be 0 or 1");
        c->ph.emission_gather = uint32_t(value);
        return LBM_OK;
    }
    return fail(c, LBM_EINVAL, "unknown tunable");
}

lbm_status lbm_get_tunable(const lbm_ctx *c, int32_t which, int64_t *value) {
    if (!c || !value) return LBM_EINVAL;
    if (c->lattice == LBM_LATTICE_D2Q9) return LBM_EUNSUPPORTED;
    if (which == LBM_TUNE_YTILE) {
        *value = c->ytile;
        return LBM_OK;
    }
    if (which == LBM_TUNE_SWEEP) {
        *value = c->compact;
        return LBM_OK;
    }
    if (which == LBM_TUNE_EMISSION) {
        *value = c->ph.emission_gather;
        return LBM_OK;
    }
    return LBM_EINVAL;
}

lbm_status lbm_set_timing(lbm_ctx *c, int32_t enable) {
    if (!c) return LBM_EINVAL;
    if (c->lattice == LBM_LATTICE_D2Q9) return plane_unsupported(c, "lbm_set_timing");
    if (enable < 0 || enable > 2) return fail(c, LBM_EINVAL, "timing must be 0, 1 or 2");
    if (enable && c->ring.empty()) {
        c->ring.resize(TIMING_RING);
        for (auto &r : c->ring) {
            r.pending = false;
            r.flushed = false;
            for (auto &ev : r.ev) {
                hipError_t e = hipEventCreate(&ev);
                if (e != hipSuccess) return hip_fail(c, e, "event create");
            }
        }
    }
    if (enable) {
        for (auto &r : c->ring) r.pending = false;
        c->times = lbm_kernel_times_t{};
    }
    c->timing = enable;
    return LBM_OK;
}

lbm_status lbm_kernel_times(lbm_ctx *c, lbm_kernel_times_t *t) {
    if (!c || !t) return LBM_EINVAL;
    if (c->lattice == LBM_LATTICE_D2Q9) return plane_unsupported(c, "lbm_kernel_times");
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "synchronize");
    for (auto &r : c->ring) drain_slot(c, r);
    *t = c->times;
    return LBM_OK;
}

namespace {
constexpr int NPARAMS = 21;

struct CkptHeader {
    uint64_t magic;
    int64_t nx, ny, nz, storage, step, nfluid, niface, nfp, cur;
    uint64_t geom_hash;
    double params[NPARAMS];
    DevTotals tot;
};

void pack_params(const lbm_ctx *c, double *p) {
    std::memset(p, 0, NPARAMS * sizeof(double));
    p[0] = c->ph.tau_gas;
    p[1] = c->ph.tau_species;
    p[2] = c->ph.force[0];
    p[3] = c->ph.force[1];
    p[4] = c->ph.force[2];
    p[5] = c->ph.rho_ref;
    p[6] = c->ph.c_ref;
    p[7] = c->ph.rho0;
    p[8] = c->ph.c0;
    p[9] = c->ph.c_inlet;
    p[10] = c->ph.p_stick;
    p[11] = c->ph.p;
    p[12] = c->ph.sputter;
    p[13] = c->ph.coupling;
    p[14] = c->ph.species_x;
    p[15] = c->ph.product;
    p[16] = c->ph.p_stick_product;
    // the STOCHASTIC key, bit for bit (the checks compare bytes)
    std::memcpy(&p[17], &c->ph.seed, sizeof(uint64_t));
    p[18] = c->ph.wall_diffuse;
    // 16-bit storage: the rounding of the stores (FP32 and FP64 ignore it)
    p[19] = storage_bytes(c->ph.storage) == 2 ? c->ph.rounding : 0;
    p[20] = c->ph.store_ux;  // the stored carrier values depend on it
}

// Product-lattice bytes of a checkpoint: P buffers A and B, E_P, Acc_P.
size_t ckpt_product_bytes(const lbm_ctx *c) {
    if (!c->ph.product) return 0;
    const size_t sb = size_t(storage_bytes(c->ph.storage));
    return size_t(38) * c->nfp * sb + size_t(c->niface) * sb + size_t(c->niface) * 8;
}
}  // namespace

lbm_status lbm_save(lbm_ctx *c, const char *path) {
    if (!c || !path) return fail(c, LBM_EINVAL, "NULL argument");
    if (c->lattice == LBM_LATTICE_D2Q9) return plane_unsupported(c, "lbm_save");
    CkptHeader h{};
    h.magic = CKPT_MAGIC;
    h.nx = c->nx;
    h.ny = c->ny;
    h.nz = c->nz;
    h.storage = c->ph.storage;
    h.step = c->step;
    h.nfluid = c->nfluid;
    h.niface = c->niface;
    h.nfp = c->nfp;
    h.cur = c->cur;
    h.geom_hash = c->geom_hash;
    pack_params(c, h.params);
    hipError_t e = hipMemcpyAsync(&h.tot, c->d_tot, sizeof(DevTotals), hipMemcpyDeviceToHost, c->stream);
    const size_t pop = size_t(38) * c->nfp * storage_bytes(c->ph.storage);
    const size_t emit = size_t(nslot(c) * c->niface) * storage_bytes(c->ph.storage);
    const size_t base = 2 * pop + emit + size_t(c->niface) * 8, pbytes = ckpt_product_bytes(c);
    std::vector<char> buf;
    try {
        buf.resize(base + pbytes);
    } catch (const std::bad_alloc &) {
        return fail(c, LBM_ENOMEM, "checkpoint buffer");
    }
    if (e == hipSuccess) e = hipMemcpyAsync(buf.data(), c->d_pop[0], pop, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(buf.data() + pop, c->d_pop[1], pop, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(buf.data() + 2 * pop, c->d_emit, emit, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && c->niface)
        e = hipMemcpyAsync(buf.data() + 2 * pop + emit, c->d_acc, size_t(c->niface) * 8, hipMemcpyDeviceToHost,
                           c->stream);
    if (e == hipSuccess && pbytes) {
        // d_popP[0], d_popP[1] and E_P are one contiguous block
        const size_t pe = pbytes - size_t(c->niface) * 8;
        e = hipMemcpyAsync(buf.data() + base, c->d_popP[0], pe, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess && c->niface)
            e = hipMemcpyAsync(buf.data() + base + pe, c->d_accP, size_t(c->niface) * 8, hipMemcpyDeviceToHost,
                               c->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "checkpoint copy");
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(c, LBM_EINVAL, std::string("cannot open ") + path);
    const bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1 && std::fwrite(buf.data(), 1, buf.size(), f) == buf.size();
    if (std::fclose(f) != 0 || !ok) return fail(c, LBM_EINVAL, std::string("write failed: ") + path);
    return LBM_OK;
}

lbm_status lbm_load(lbm_ctx *c, const char *path) {
    if (!c || !path) return fail(c, LBM_EINVAL, "NULL argument");
    if (c->lattice == LBM_LATTICE_D2Q9) return plane_unsupported(c, "lbm_load");
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(c, LBM_EINVAL, std::string("cannot open ") + path);
    CkptHeader h{};
    if (std::fread(&h, sizeof(h), 1, f) != 1 || h.magic != CKPT_MAGIC) {
        std::fclose(f);
        return fail(c, LBM_EINVAL, "not a checkpoint of this library");
    }
    double params[NPARAMS];
    pack_params(c, params);
    if (h.nx != c->nx || h.ny != c->ny || h.nz != c->nz || h.storage != c->ph.storage || h.nfluid != c->nfluid ||
        h.niface != c->niface || h.nfp != c->nfp || h.geom_hash != c->geom_hash ||
        std::memcmp(params, h.params, sizeof(params)) != 0) {
        std::fclose(f);
        return fail(c, LBM_EINVAL, "checkpoint does not match this context's geometry or parameters");
    }
    const size_t pop = size_t(38) * c->nfp * storage_bytes(c->ph.storage);
    const size_t emit = size_t(nslot(c) * c->niface) * storage_bytes(c->ph.storage);
    const size_t base = 2 * pop + emit + size_t(c->niface) * 8, pbytes = ckpt_product_bytes(c);
    std::vector<char> buf;
    try {
        buf.resize(base + pbytes);
    } catch (const std::bad_alloc &) {
        std::fclose(f);
        return fail(c, LBM_ENOMEM, "checkpoint buffer");
    }
    const bool ok = std::fread(buf.data(), 1, buf.size(), f) == buf.size();
    std::fclose(f);
    if (!ok) return fail(c, LBM_EINVAL, "truncated checkpoint");
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->d_pop[0], buf.data(), pop, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->d_pop[1], buf.data() + pop, pop, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->d_emit, buf.data() + 2 * pop, emit, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && c->niface)
        e = hipMemcpyAsync(c->d_acc, buf.data() + 2 * pop + emit, size_t(c->niface) * 8, hipMemcpyHostToDevice,
                           c->stream);
    if (e == hipSuccess && pbytes) {
        const size_t pe = pbytes - size_t(c->niface) * 8;
        e = hipMemcpyAsync(c->d_popP[0], buf.data() + base, pe, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess && c->niface)
            e = hipMemcpyAsync(c->d_accP, buf.data() + base + pe, size_t(c->niface) * 8, hipMemcpyHostToDevice,
                               c->stream);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(c->d_tot, &h.tot, sizeof(DevTotals), hipMemcpyHostToDevice, c->stream);
    c->step = h.step;
    c->cur = int(h.cur);
    c->ph.step_ctr = uint32_t(c->step);
    // In(k) of the pending interface is derived state: rebuild it from the
    // current post-collision populations (the same integer terms the sweep adds)
    if (e == hipSuccess) e = launch_in_init(geometry(c), c->ph, interface_list(c), c->d_pop[c->cur], c->stream);
    if (e == hipSuccess && c->ph.product)
        e = launch_in_init_product(geometry(c), c->ph, interface_list(c), c->d_popP[c->cur], c->d_inaccP, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "checkpoint upload");
    c->flag_pending = false;
    *c->h_flag = h.tot.nonfinite;
    return LBM_OK;
}

// Autotuner: time the sweep for every candidate (sweep variant x y-tile)
// in place, then restore what the trial sweeps overwrote.  A sweep reads the
// current post-collision buffer and the emission array and writes only the
// other population buffer, the In(k) accumulators and its partial sums, so saving
// and restoring the first two leaves the state exactly as it was.
}  // extern "C"

namespace {

struct Candidate {
    int compact, ytile, gather;
};

// Sweep variant x y-tile, and for the compact sweep both emission read modes
// where the gather applies (`gather_ok`); elsewhere the candidates keep the
// current mode `gather_now`, which has no effect there.
std::vector<Candidate> tuning_candidates(bool compact_ok, int ny, bool compact_only, bool gather_ok, int gather_now) {
    std::vector<Candidate> out;
    const int ytiles[] = {4, 8, 16, 32, 64, 128};
    for (int v = compact_only ? 1 : 0; v <= (compact_ok ? 1 : 0); ++v) {
        const bool both = v == 1 && gather_ok;
        for (int gm = both ? 0 : gather_now; gm <= (both ? 1 : gather_now); ++gm) {
            int last = -1;
            for (int yt : ytiles) {
                const int t = std::min(yt, ny);
                if (t == last) continue;
                out.push_back({v, t, gm});
                last = t;
            }
        }
    }
    return out;
}

struct Saved {
    void *pop = nullptr, *link = nullptr;    // saved population buffer and In(k) accumulators
    void *popP = nullptr, *linkP = nullptr;  // the same of the product lattice
};

lbm_status save_written(lbm_ctx *c, Saved &sv, void *(*alloc)(lbm_ctx *, size_t)) {
    const size_t pop = size_t(38) * c->nfp * storage_bytes(c->ph.storage);
    const size_t link = size_t(nslot(c) * c->niface) * 8;
    sv.pop = alloc(c, pop);
    sv.link = alloc(c, std::max<size_t>(link, 256));
    if (!sv.pop || !sv.link) return fail(c, LBM_ENOMEM, "autotune scratch allocation failed");
    if (c->ph.product) {
        sv.popP = alloc(c, pop / 2);
        sv.linkP = alloc(c, std::max<size_t>(link, 256));
        if (!sv.popP || !sv.linkP) return fail(c, LBM_ENOMEM, "autotune scratch allocation failed");
    }
    hipError_t e = hipMemcpyAsync(sv.pop, c->d_pop[1 - c->cur], pop, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess && link) e = hipMemcpyAsync(sv.link, c->d_inacc, link, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess && c->ph.product)
        e = hipMemcpyAsync(sv.popP, c->d_popP[1 - c->cur], pop / 2, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess && c->ph.product && link)
        e = hipMemcpyAsync(sv.linkP, c->d_inaccP, link, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "autotune save");
    return LBM_OK;
}

lbm_status restore_written(lbm_ctx *c, Saved &sv) {
    const size_t pop = size_t(38) * c->nfp * storage_bytes(c->ph.storage);
    const size_t link = size_t(nslot(c) * c->niface) * 8;
    hipError_t e = hipMemcpyAsync(c->d_pop[1 - c->cur], sv.pop, pop, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess && link) e = hipMemcpyAsync(c->d_inacc, sv.link, link, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess && sv.popP)
        e = hipMemcpyAsync(c->d_popP[1 - c->cur], sv.popP, pop / 2, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess && sv.linkP && link)
        e = hipMemcpyAsync(c->d_inaccP, sv.linkP, link, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "autotune restore");
    return LBM_OK;
}

void *scratch_alloc(lbm_ctx *c, size_t bytes) {
    void *p = nullptr;
    if (c->dev.alloc)
        p = c->dev.alloc(bytes, c->dev.user);
    else if (hipMalloc(&p, bytes) != hipSuccess)
        p = nullptr;
    return p;
}

void scratch_free(lbm_ctx *c, void *p) {
    if (!p) return;
    if (c->dev.free)
        c->dev.free(p, c->dev.user);
    else
        (void)hipFree(p);
}

// Mean time of `reps` launches of `launch` (after one untimed launch).
template <typename F>
lbm_status time_launches(hipStream_t s, int reps, F &&launch, float *ms, std::string *err) {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(a, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e != hipSuccess) {
        *err = std::string("autotune timing: ") + hipGetErrorString(e);
        return LBM_EDEVICE;
    }
    *ms /= float(reps);
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_autotune(lbm_ctx *c, int32_t reps, double *best_ms) {
    if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
    if (c->lattice == LBM_LATTICE_D2Q9) return plane_unsupported(c, "lbm_autotune");
    if (reps < 1 || reps > 1000) return fail(c, LBM_EINVAL, "reps must be in [1, 1000]");
    lbm_status st = check_pending_flag(c);
    if (st != LBM_OK) return st;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "autotune");
    Saved sv;
    st = save_written(c, sv, scratch_alloc);
    const Candidate keep{c->compact, c->ytile, int(c->ph.emission_gather)};
    Candidate best = keep;
    float best_t = 0.0f;
    const std::vector<Candidate> cands =
        tuning_candidates(c->compact_ok, c->ny, c->ph.product != 0,
                          emission_gather_applies(c->ph.storage, c->ph.sputter, c->ph.product != 0), keep.gather);
    std::vector<float> t_min(cands.size(), 0.0f);
    // two interleaved rounds; each candidate keeps its faster round
    for (int round = 0; round < 2 && st == LBM_OK; ++round) {
        for (size_t ci = 0; ci < cands.size(); ++ci) {
            const Candidate &cd = cands[ci];
            st = lbm_set_tunable(c, LBM_TUNE_YTILE, cd.ytile);
            if (st == LBM_OK) st = lbm_set_tunable(c, LBM_TUNE_SWEEP, cd.compact);
            if (st == LBM_OK) st = lbm_set_tunable(c, LBM_TUNE_EMISSION, cd.gather);
            if (st != LBM_OK) break;
            const Geometry g = geometry(c);
            const void *fin = c->d_pop[c->cur];
            void *fout = c->d_pop[1 - c->cur];
            float ms = 0.0f;
            ProdStep pst = c->ph.product ? prod_step(c, c->step) : ProdStep{};
            const ProdStep *prod = c->ph.product ? &pst : nullptr;
            c->ph.step_ctr = uint32_t(c->step + 1);
            st = time_launches(c->stream, reps, [&]() {
                return c->compact ? launch_sweep_c(g, c->ph, fin, fout, c->d_emit, c->d_part, c->stream, prod)
                                  : launch_sweep(g, c->ph, fin, fout, c->d_emit, c->d_part, c->stream);
            }, &ms, &c->err);
            if (st != LBM_OK) break;
            if (round == 0 || ms < t_min[ci]) t_min[ci] = ms;
        }
    }
    for (size_t ci = 0; ci < cands.size() && st == LBM_OK; ++ci)
        if (best_t == 0.0f || t_min[ci] < best_t) {
            best_t = t_min[ci];
            best = cands[ci];
        }
    lbm_status rs = sv.pop ? restore_written(c, sv) : LBM_OK;
    scratch_free(c, sv.pop);
    scratch_free(c, sv.link);
    scratch_free(c, sv.popP);
    scratch_free(c, sv.linkP);
    const Candidate use = st == LBM_OK ? best : keep;
    lbm_status ts = lbm_set_tunable(c, LBM_TUNE_YTILE, use.ytile);
    if (ts == LBM_OK) ts = lbm_set_tunable(c, LBM_TUNE_SWEEP, use.compact);
    if (ts == LBM_OK) ts = lbm_set_tunable(c, LBM_TUNE_EMISSION, use.gather);
    if (st != LBM_OK) return st;
    if (rs != LBM_OK) return rs;
    if (ts != LBM_OK) return ts;
    if (best_ms) *best_ms = double(best_t);
    return LBM_OK;
}

const char *lbm_last_error(const lbm_ctx *c) { return c ? c->err.c_str() : g_create_error.c_str(); }

void lbm_destroy(lbm_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    release(c);
    delete c;
}

// ---------------------------------------------------------------------------
// Batches

struct lbm_batch {
    std::vector<lbm_ctx *> ctx;
    lbm_device dev{};
    hipStream_t stream = nullptr;
    int storage = 0, sputter = 0, species_x = 0;  // shared by every sample
    bool compact = false;  // node-compact sweep for every sample (all support it)
    // emission reads of the compact sweep gathered through LDS where that
    // applies (LBM_TUNE_EMISSION); direct by default, measured faster on the
    // 64-sample batch
    bool gather = false;
    std::vector<void *> allocations;
    void *d_records = nullptr;
    ReduceK *d_reduce = nullptr;
    uint32_t *d_sweep_sample = nullptr, *d_iface_sample = nullptr;
    int64_t sweep_blocks_total = 0, iface_blocks_total = 0;
    int parity = 0;
    bool use_graph = false;
    hipStream_t capture = nullptr;
    // captured step loops starting at buffer parity 0 / 1: [0] two steps,
    // [1] LONG_GRAPH_STEPS steps (both even, so a replay keeps the parity)
    hipGraph_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    hipGraphExec_t exec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    // sweep timing (lbm_batch_set_timing): one start/stop event pair per
    // eager step in a ring, drained into ms_sweep / n_sweep
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ring;
    std::vector<bool> ring_pending;
    int ring_next = 0;
    double ms_sweep = 0.0;
    int64_t n_sweep = 0;
    std::string err;
};

// Steps of the long captured loop: replays of it carry a batch's runs of
// many steps with one graph launch per 64 steps.
constexpr int64_t LONG_GRAPH_STEPS = 64;

namespace {

thread_local std::string g_batch_create_error;

lbm_status bfail(lbm_batch *b, lbm_status s, const std::string &msg) {
    if (b)
        b->err = msg;
    else
        g_batch_create_error = msg;
    return s;
}

void batch_release(lbm_batch *b) {
    if (b->stream || !b->ctx.empty()) (void)hipStreamSynchronize(b->stream);
    for (auto &ev : b->ring) {
        if (ev.first) (void)hipEventDestroy(ev.first);
        if (ev.second) (void)hipEventDestroy(ev.second);
    }
    b->ring.clear();
    b->ring_pending.clear();
    for (int l = 0; l < 2; ++l)
        for (int k = 0; k < 2; ++k) {
            if (b->exec[l][k]) (void)hipGraphExecDestroy(b->exec[l][k]);
            if (b->graph[l][k]) (void)hipGraphDestroy(b->graph[l][k]);
        }
    if (b->capture) (void)hipStreamDestroy(b->capture);
    for (void *p : b->allocations) {
        if (b->dev.free)
            b->dev.free(p, b->dev.user);
        else
            (void)hipFree(p);
    }
    b->allocations.clear();
    for (lbm_ctx *c : b->ctx) lbm_destroy(c);
    b->ctx.clear();
}

void *batch_alloc(lbm_batch *b, size_t bytes) {
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (b->dev.alloc)
        p = b->dev.alloc(bytes, b->dev.user);
    else if (hipMalloc(&p, bytes) != hipSuccess)
        p = nullptr;
    if (p) b->allocations.push_back(p);
    return p;
}

void batch_drain(lbm_batch *b, size_t k) {
    if (!b->ring_pending[k]) return;
    float ms = 0.0f;
    (void)hipEventSynchronize(b->ring[k].second);
    if (hipEventElapsedTime(&ms, b->ring[k].first, b->ring[k].second) == hipSuccess) {
        b->ms_sweep += ms;
        b->n_sweep += 1;
    }
    b->ring_pending[k] = false;
}

lbm_status batch_launch(lbm_batch *b, int parity, hipStream_t s, bool timed = false) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
        const size_t k = size_t(b->ring_next);
        b->ring_next = (b->ring_next + 1) % int(b->ring.size());
        batch_drain(b, k);
        e0 = b->ring[k].first;
        e1 = b->ring[k].second;
        b->ring_pending[k] = true;
    }
    hipError_t e = launch_batch_step(b->storage, b->sputter, b->species_x, b->compact, b->gather, b->d_records,
                                     b->d_sweep_sample,
                                     b->sweep_blocks_total, b->d_iface_sample, b->iface_blocks_total, b->d_reduce,
                                     int(b->ctx.size()), parity, s, e0, e1);
    if (e != hipSuccess) return bfail(b, e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE,
                                      std::string("batch step launch: ") + hipGetErrorString(e));
    return LBM_OK;
}

// Capture `steps` (even) consecutive steps starting at buffer parity
// `parity` on a private stream, as loop `l` (0: two steps, 1: the long
// loop); the executable graph is later launched on the batch stream.
lbm_status batch_capture(lbm_batch *b, int l, int parity, int64_t steps) {
    hipError_t e = hipSuccess;
    if (!b->capture) e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bfail(b, LBM_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    lbm_status st = LBM_OK;
    for (int64_t k = 0; k < steps && st == LBM_OK; ++k) st = batch_launch(b, int((parity + k) & 1), b->capture);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->capture, &g);
    if (st != LBM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec[l][parity], g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        b->exec[l][parity] = nullptr;
        return bfail(b, LBM_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    b->graph[l][parity] = g;
    return LBM_OK;
}

lbm_status batch_sample(lbm_batch *b, int32_t i, lbm_ctx **c) {
    if (!b) return LBM_EINVAL;
    if (i < 0 || size_t(i) >= b->ctx.size()) return bfail(b, LBM_EINVAL, "sample index out of range");
    *c = b->ctx[size_t(i)];
    return LBM_OK;
}

lbm_status batch_forward(lbm_batch *b, int32_t i, lbm_status st) {
    if (st != LBM_OK) b->err = "sample " + std::to_string(i) + ": " + b->ctx[size_t(i)]->err;
    return st;
}

// Per-sample block ranges (samples in order, each with its single-sample
// block count for the batch's sweep variant), the block-to-sample tables and
// the device records; every context is switched to the batch's variant so a
// sample's single-context calls match its batched steps.
// Destroy the captured step graphs (they hold the launches as captured).
void drop_graphs(lbm_batch *b) {
    for (int l = 0; l < 2; ++l)
        for (int k = 0; k < 2; ++k) {
            if (b->exec[l][k]) (void)hipGraphExecDestroy(b->exec[l][k]);
            if (b->graph[l][k]) (void)hipGraphDestroy(b->graph[l][k]);
            b->exec[l][k] = nullptr;
            b->graph[l][k] = nullptr;
        }
}

lbm_status batch_tables(lbm_batch *b) {
    const int n = int(b->ctx.size());
    for (lbm_ctx *c : b->ctx) c->compact = b->compact ? 1 : 0;
    std::vector<BatchSample> smp(static_cast<size_t>(n));
    std::vector<ReduceK> red(static_cast<size_t>(n));
    int64_t nb = 0, ni = 0;
    for (int i = 0; i < n; ++i) {
        lbm_ctx *c = b->ctx[size_t(i)];
        BatchSample &s = smp[size_t(i)];
        s.g = geometry(c);
        s.it = interface_list(c);
        s.ph = c->ph;
        s.pop[0] = c->d_pop[0];
        s.pop[1] = c->d_pop[1];
        s.emit = c->d_emit;
        s.part_sweep = c->d_part;
        s.part_iface = part_iface(c, 0);
        s.block0 = uint32_t(nb);
        s.iblock0 = uint32_t(ni);
        nb += active_sweep_blocks(c);
        ni += c->blocks_iface;
        ReduceK &r = red[size_t(i)];
        r.ps = s.part_sweep;
        r.ns = active_sweep_blocks(c);
        r.pi = s.part_iface;
        r.ni = c->blocks_iface;
        r.fold = part_fold(c, 0);
        r.p = c->ph.p;
        r.p_stick = c->ph.p_stick;
        r.tot = c->d_tot;
    }
    b->sweep_blocks_total = nb;
    b->iface_blocks_total = ni;
    std::vector<uint32_t> sweep_sample(size_t(std::max<int64_t>(nb, 1))), iface_sample(size_t(std::max<int64_t>(ni, 1)));
    for (int i = 0; i < n; ++i) {
        const lbm_ctx *c = b->ctx[size_t(i)];
        std::fill_n(sweep_sample.begin() + smp[size_t(i)].block0, active_sweep_blocks(c), uint32_t(i));
        std::fill_n(iface_sample.begin() + smp[size_t(i)].iblock0, c->blocks_iface, uint32_t(i));
    }
    hipError_t e = hipStreamSynchronize(b->stream);  // earlier steps may still read the tables
    if (e == hipSuccess) e = batch_upload(b->storage, smp.data(), n, b->d_records, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_reduce, red.data(), red.size() * sizeof(ReduceK), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_sweep_sample, sweep_sample.data(), sweep_sample.size() * 4, hipMemcpyHostToDevice,
                           b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_iface_sample, iface_sample.data(), iface_sample.size() * 4, hipMemcpyHostToDevice,
                           b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, LBM_EDEVICE, std::string("batch upload: ") + hipGetErrorString(e));
    drop_graphs(b);  // captured graphs hold the old launch shapes
    return LBM_OK;
}

}  // namespace

lbm_status lbm_batch_create(int32_t n, const lbm_geometry *g, const double *kn, const double *da,
                            const double (*tau)[2], const lbm_bc *bc, const lbm_device *dev, lbm_batch **out) {
    if (!out) return bfail(nullptr, LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1) return bfail(nullptr, LBM_EINVAL, "a batch needs n >= 1 samples");
    if (!g || !da || !tau || !bc) return bfail(nullptr, LBM_EINVAL, "g, da, tau and bc must not be NULL");
    for (int32_t i = 0; i < n; ++i)
        if (bc[i].product != 0)
            return bfail(nullptr, LBM_EUNSUPPORTED, "the product lattice is not available in batches");
        else if (bc[i].sputter == LBM_SPUTTER_STOCHASTIC)
            return bfail(nullptr, LBM_EUNSUPPORTED, "STOCHASTIC sputtering is not available in batches");
        else if (bc[i].wall_diffuse != 0.0 || bc[i].wall_accommodation != 0.0)
            return bfail(nullptr, LBM_EUNSUPPORTED, "the diffuse wall is not available in batches");
        else if (bc[i].lattice != LBM_LATTICE_D3Q19)
            return bfail(nullptr, LBM_EUNSUPPORTED, "batches take D3Q19 samples only");
        else if (bc[i].rounding == LBM_ROUND_STOCHASTIC && (bc[i].storage == LBM_STORE_F16 ||
                                                           bc[i].storage == LBM_STORE_BF16))
            // a captured batch graph replays the launch arguments, and with
            // them the step key of the rounding words
            return bfail(nullptr, LBM_EUNSUPPORTED, "stochastic rounding is not available in batches");
    for (int32_t i = 1; i < n; ++i)
        if (bc[i].storage != bc[0].storage || bc[i].sputter != bc[0].sputter || bc[i].coupling != bc[0].coupling ||
            bc[i].species_x != bc[0].species_x)
            return bfail(nullptr, LBM_EINVAL,
                         "sample " + std::to_string(i) + ": storage, sputter, coupling and species_x must match sample 0");
    lbm_batch *b = new (std::nothrow) lbm_batch();
    if (!b) return bfail(nullptr, LBM_ENOMEM, "host allocation failed");
    if (dev) b->dev = *dev;
    b->stream = static_cast<hipStream_t>(b->dev.stream);
    b->storage = bc[0].storage;
    b->sputter = bc[0].sputter;
    b->species_x = bc[0].species_x;
    try {
        b->ctx.reserve(size_t(n));
        for (int32_t i = 0; i < n; ++i) {
            lbm_ctx *c = nullptr;
            lbm_status st = lbm_create_on(&g[i], kn ? kn[i] : 0.0, da[i], tau[i], &bc[i], dev, &c);
            if (st != LBM_OK) {
                std::string msg = "sample " + std::to_string(i) + ": " + g_create_error;
                batch_release(b);
                delete b;
                return bfail(nullptr, st, msg);
            }
            b->ctx.push_back(c);
        }
        // One sweep variant for all samples: node-compact if every sample
        // supports it.
        b->compact = true;
        for (lbm_ctx *c : b->ctx) b->compact = b->compact && c->compact_ok;
        int64_t nb_max = 0, ni = 0;
        for (lbm_ctx *c : b->ctx) {
            nb_max += c->part_rows;  // the larger sweep variant's block count
            ni += c->blocks_iface;
        }
        if (nb_max >= (int64_t(1) << 31) || ni >= (int64_t(1) << 31)) {
            batch_release(b);
            delete b;
            return bfail(nullptr, LBM_EINVAL, "batch too large for one launch");
        }
        b->d_records = batch_alloc(b, batch_record_bytes(b->storage) * size_t(n));
        b->d_reduce = static_cast<ReduceK *>(batch_alloc(b, sizeof(ReduceK) * size_t(n)));
        b->d_sweep_sample = static_cast<uint32_t *>(batch_alloc(b, size_t(std::max<int64_t>(nb_max, 1)) * 4));
        b->d_iface_sample = static_cast<uint32_t *>(batch_alloc(b, size_t(std::max<int64_t>(ni, 1)) * 4));
        if (!b->d_records || !b->d_reduce || !b->d_sweep_sample || !b->d_iface_sample) {
            batch_release(b);
            delete b;
            return bfail(nullptr, LBM_ENOMEM, "device allocation failed");
        }
        const lbm_status st = batch_tables(b);
        if (st != LBM_OK) {
            std::string msg = b->err;
            batch_release(b);
            delete b;
            return bfail(nullptr, st, msg);
        }
    } catch (const std::bad_alloc &) {
        batch_release(b);
        delete b;
        return bfail(nullptr, LBM_ENOMEM, "host allocation failed");
    }
    *out = b;
    return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch *b, int64_t n) {
    if (!b) return LBM_EINVAL;
    if (n < 0) return bfail(b, LBM_EINVAL, "n must be >= 0");
    for (size_t i = 0; i < b->ctx.size(); ++i) {
        const lbm_status st = check_pending_flag(b->ctx[i]);
        if (st != LBM_OK) return batch_forward(b, int32_t(i), st);
    }
    int64_t done = 0;
    lbm_status failed = LBM_OK;
    if (b->use_graph && !b->timing) {
        // the long loop while at least LONG_GRAPH_STEPS remain, then two-step loops
        for (int l = 1; l >= 0 && failed == LBM_OK; --l) {
            const int64_t len = l ? LONG_GRAPH_STEPS : 2;
            while (done + len <= n) {
                if (!b->exec[l][b->parity]) {
                    failed = batch_capture(b, l, b->parity, len);
                    if (failed != LBM_OK) break;
                }
                const hipError_t e = hipGraphLaunch(b->exec[l][b->parity], b->stream);
                if (e != hipSuccess) {
                    failed = bfail(b, LBM_EDEVICE, std::string("graph launch: ") + hipGetErrorString(e));
                    break;
                }
                done += len;
            }
        }
    }
    for (; failed == LBM_OK && done < n; ++done) {
        failed = batch_launch(b, b->parity, b->stream, b->timing);
        if (failed != LBM_OK) break;
        b->parity = 1 - b->parity;
    }
    n = done;  // the steps actually queued
    // graph replays (even step counts) leave the parity unchanged; the per-sample
    // contexts track the same parity and step count
    for (lbm_ctx *c : b->ctx) {
        c->cur = b->parity;
        c->step += n;
    }
    if (n > 0) {
        for (size_t i = 0; i < b->ctx.size(); ++i) {
            lbm_ctx *c = b->ctx[i];
            hipError_t e = hipMemcpyAsync(c->h_flag, &c->d_tot->nonfinite, sizeof(int32_t), hipMemcpyDeviceToHost,
                                          b->stream);
            if (e == hipSuccess) e = hipEventRecord(c->flag_event, b->stream);
            if (e != hipSuccess) return bfail(b, LBM_EDEVICE, std::string("watchdog copy: ") + hipGetErrorString(e));
            c->flag_pending = true;
        }
    }
    return failed;
}

lbm_status lbm_batch_set_timing(lbm_batch *b, int32_t enable) {
    if (!b) return LBM_EINVAL;
    if (enable != 0 && enable != 2) return bfail(b, LBM_EINVAL, "batch timing must be 0 or 2 (the sweep)");
    if (enable && b->ring.empty()) {
        b->ring.assign(TIMING_RING, {nullptr, nullptr});
        b->ring_pending.assign(TIMING_RING, false);
        for (auto &ev : b->ring) {
            hipError_t e = hipEventCreate(&ev.first);
            if (e == hipSuccess) e = hipEventCreate(&ev.second);
            if (e != hipSuccess) return bfail(b, LBM_EDEVICE, std::string("event create: ") + hipGetErrorString(e));
        }
    }
    if (enable) {
        std::fill(b->ring_pending.begin(), b->ring_pending.end(), false);
        b->ms_sweep = 0.0;
        b->n_sweep = 0;
    }
    b->timing = enable != 0;
    return LBM_OK;
}

lbm_status lbm_batch_kernel_times(lbm_batch *b, lbm_kernel_times_t *t) {
    if (!b || !t) return LBM_EINVAL;
    const hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, LBM_EDEVICE, std::string("synchronize: ") + hipGetErrorString(e));
    for (size_t k = 0; k < b->ring.size(); ++k) batch_drain(b, k);
    *t = lbm_kernel_times_t{};
    t->ms_sweep = b->ms_sweep;
    t->n_sweep = b->n_sweep;
    return LBM_OK;
}

lbm_status lbm_batch_fields(lbm_batch *b, int32_t i, double *rho, double *u, double *conc) {
    lbm_ctx *c = nullptr;
    lbm_status st = batch_sample(b, i, &c);
    return st != LBM_OK ? st : batch_forward(b, i, lbm_fields(c, rho, u, conc));
}

lbm_status lbm_batch_conversion_map(lbm_batch *b, int32_t i, double *conv) {
    lbm_ctx *c = nullptr;
    lbm_status st = batch_sample(b, i, &c);
    return st != LBM_OK ? st : batch_forward(b, i, lbm_conversion_map(c, conv));
}

lbm_status lbm_batch_totals(lbm_batch *b, int32_t i, lbm_totals_t *t) {
    lbm_ctx *c = nullptr;
    lbm_status st = batch_sample(b, i, &c);
    return st != LBM_OK ? st : batch_forward(b, i, lbm_totals(c, t));
}

lbm_status lbm_batch_query(const lbm_batch *b, int32_t i, lbm_info *info) {
    if (!b || i < 0 || size_t(i) >= b->ctx.size()) return LBM_EINVAL;
    return lbm_query(b->ctx[size_t(i)], info);
}

lbm_status lbm_batch_synchronize(lbm_batch *b) {
    if (!b) return LBM_EINVAL;
    const hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, LBM_EDEVICE, std::string("synchronize: ") + hipGetErrorString(e));
    for (size_t i = 0; i < b->ctx.size(); ++i) {
        const lbm_status st = check_pending_flag(b->ctx[i]);
        if (st != LBM_OK) return batch_forward(b, int32_t(i), st);
    }
    return LBM_OK;
}

lbm_status lbm_batch_set_graph(lbm_batch *b, int32_t enable) {
    if (!b) return LBM_EINVAL;
    if (enable != 0 && enable != 1) return bfail(b, LBM_EINVAL, "enable must be 0 or 1");
    b->use_graph = enable == 1;
    return LBM_OK;
}

lbm_status lbm_batch_set_tunable(lbm_batch *b, int32_t which, int64_t value) {
    if (!b) return LBM_EINVAL;
    if (which == LBM_TUNE_SWEEP) {
        if (value != 0 && value != 1) return bfail(b, LBM_EINVAL, "sweep variant must be 0 or 1");
        if (value == 1)
            for (const lbm_ctx *c : b->ctx)
                if (!c->compact_ok) return bfail(b, LBM_EUNSUPPORTED, "a sample does not support the compact sweep");
        b->compact = value == 1;
        return batch_tables(b);
    }
    if (which == LBM_TUNE_EMISSION) {
        if (value != 0 && value != 1) return bfail(b, LBM_EINVAL, "emission read mode must be 0 or 1");
        if (b->gather != (value == 1)) {
            // the stream may still replay a graph that holds the old launch
            const hipError_t e = hipStreamSynchronize(b->stream);
            if (e != hipSuccess) return bfail(b, LBM_EDEVICE, std::string("set tunable: ") + hipGetErrorString(e));
            drop_graphs(b);
            b->gather = value == 1;
        }
        return LBM_OK;
    }
    if (which == LBM_TUNE_YTILE) {
        if (value < 1) return bfail(b, LBM_EINVAL, "ytile must be >= 1");
        for (size_t i = 0; i < b->ctx.size(); ++i) {
            lbm_ctx *c = b->ctx[i];
            const lbm_status st = lbm_set_tunable(c, LBM_TUNE_YTILE, std::min<int64_t>(value, c->ny));
            if (st != LBM_OK) return batch_forward(b, int32_t(i), st);
        }
        return LBM_OK;
    }
    return bfail(b, LBM_EINVAL, "unknown tunable");
}

lbm_status lbm_batch_get_tunable(const lbm_batch *b, int32_t which, int64_t *value) {
    if (!b || !value || b->ctx.empty()) return LBM_EINVAL;
    if (which == LBM_TUNE_SWEEP) {
        *value = b->compact ? 1 : 0;
        return LBM_OK;
    }
    if (which == LBM_TUNE_EMISSION) {
        *value = b->gather ? 1 : 0;
        return LBM_OK;
    }
    return lbm_get_tunable(b->ctx[0], which, value);
}

lbm_status lbm_batch_autotune(lbm_batch *b, int32_t reps, double *best_ms) {
    if (!b) return LBM_EINVAL;
    if (reps < 1 || reps > 1000) return bfail(b, LBM_EINVAL, "reps must be in [1, 1000]");
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, LBM_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
    for (size_t i = 0; i < b->ctx.size(); ++i) {
        const lbm_status st = check_pending_flag(b->ctx[i]);
        if (st != LBM_OK) return batch_forward(b, int32_t(i), st);
    }
    bool compact_ok = true;
    int ny_max = 1;
    for (const lbm_ctx *c : b->ctx) {
        compact_ok = compact_ok && c->compact_ok;
        ny_max = std::max(ny_max, c->ny);
    }
    std::vector<Saved> sv(b->ctx.size());
    lbm_status st = LBM_OK;
    for (size_t i = 0; i < b->ctx.size() && st == LBM_OK; ++i) {
        st = save_written(b->ctx[i], sv[i], scratch_alloc);
        if (st != LBM_OK) st = batch_forward(b, int32_t(i), st);
    }
    const Candidate keep{b->compact ? 1 : 0, b->ctx[0]->ytile, b->gather ? 1 : 0};
    Candidate best = keep;
    float best_t = 0.0f;
    const std::vector<Candidate> cands =
        tuning_candidates(compact_ok, ny_max, false,
                          emission_gather_applies(b->storage, b->sputter, b->ctx[0]->ph.product != 0), keep.gather);
    std::vector<float> t_min(cands.size(), 0.0f);
    for (int round = 0; round < 2 && st == LBM_OK; ++round) {
        for (size_t ci = 0; ci < cands.size(); ++ci) {
            const Candidate &cd = cands[ci];
            st = lbm_batch_set_tunable(b, LBM_TUNE_YTILE, cd.ytile);
            if (st == LBM_OK) st = lbm_batch_set_tunable(b, LBM_TUNE_SWEEP, cd.compact);
            if (st == LBM_OK) st = lbm_batch_set_tunable(b, LBM_TUNE_EMISSION, cd.gather);
            if (st != LBM_OK) break;
            const int parity = b->parity;
            float ms = 0.0f;
            st = time_launches(b->stream, reps, [&]() {
                return launch_batch_sweep(b->storage, b->sputter, b->species_x, b->compact, b->gather, b->d_records,
                                          b->d_sweep_sample,
                                          b->sweep_blocks_total, parity, b->stream);
            }, &ms, &b->err);
            if (st != LBM_OK) break;
            if (round == 0 || ms < t_min[ci]) t_min[ci] = ms;
        }
    }
    for (size_t ci = 0; ci < cands.size() && st == LBM_OK; ++ci)
        if (best_t == 0.0f || t_min[ci] < best_t) {
            best_t = t_min[ci];
            best = cands[ci];
        }
    lbm_status rs = LBM_OK;
    for (size_t i = 0; i < b->ctx.size(); ++i) {
        if (sv[i].pop && rs == LBM_OK) rs = restore_written(b->ctx[i], sv[i]);
        scratch_free(b->ctx[i], sv[i].pop);
        scratch_free(b->ctx[i], sv[i].link);
    }
    const Candidate use = st == LBM_OK ? best : keep;
    lbm_status ts = lbm_batch_set_tunable(b, LBM_TUNE_YTILE, use.ytile);
    if (ts == LBM_OK) ts = lbm_batch_set_tunable(b, LBM_TUNE_SWEEP, use.compact);
    if (ts == LBM_OK) ts = lbm_batch_set_tunable(b, LBM_TUNE_EMISSION, use.gather);
    if (st != LBM_OK) return st;
    if (rs != LBM_OK) return bfail(b, rs, "autotune restore failed");
    if (ts != LBM_OK) return ts;
    if (best_ms) *best_ms = double(best_t);
    return LBM_OK;
}

const char *lbm_batch_last_error(const lbm_batch *b) { return b ? b->err.c_str() : g_batch_create_error.c_str(); }

void lbm_batch_destroy(lbm_batch *b) {
    if (!b) return;
    batch_release(b);
    delete b;
}

}  // extern "C"
