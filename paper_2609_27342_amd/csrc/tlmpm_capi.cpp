// tlmpm_capi.cpp -- host runtime and C ABI of the TLMPM cutting library.
//
// Scene creation sorts the particles by reference cell (static in TLMPM: the
// reference neighbourhoods never change, Sec. III-B), builds the per-brick cell
// index, carves the caller's device workspace and uploads the state.  A substep is
// a fixed sequence of kernel launches on the caller's stream with no host
// synchronisation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tlmpm.h"
#include "tlmpm_common.h"

extern "C" {
hipError_t tl_launch_p2g(const TlLaunch*, int do_p2g, int tabs_differ, int cur, int rsb);
hipError_t tl_launch_rigid(const TlLaunch*);
hipError_t tl_launch_mixed(const TlLaunch*, int force);
hipError_t tl_launch_g2p(const TlLaunch*, int cur);
hipError_t tl_launch_labels(const TlLaunch*);
hipError_t tl_launch_slots(const TlLaunch*, int dst, int src, int force);
hipError_t tl_launch_aabb(const TlLaunch*);
hipError_t tl_launch_wrench(const TlLaunch*);
hipError_t tl_launch_resetD(const TlLaunch*);
hipError_t tl_launch_call_start(const TlLaunch*);
hipError_t tl_launch_cellmask(const TlLaunch*, int with_static, int force);
hipError_t tl_launch_cand(const TlLaunch*, int force);
hipError_t tl_launch_contact(const TlLaunch*);
hipError_t tl_launch_labels_rigid(const TlLaunch*);
hipError_t tl_launch_cand_contact_slots(const TlLaunch*, int dst, int src);
hipError_t tl_launch_fill_f32(float*, long long, float, hipStream_t);
hipError_t tl_launch_fill_i32(int*, long long, int, hipStream_t);
hipError_t tl_launch_quad(const TlLaunch*, int par, int stage);
hipError_t tl_static_scratch(int dev, void** ptr);
hipError_t tl_surface_count(const SceneK*, const SceneD*, const SurfGrid*, const SurfMem*, hipStream_t);
hipError_t tl_surface_fill(const SceneK*, const SceneD*, const SurfGrid*, const SurfMem*, hipStream_t);
hipError_t tl_surface_embed(const SceneK*, const SceneD*, const SurfMem*, int nv, hipStream_t);
}

static thread_local std::string g_err;

static tlmpm_status fail(tlmpm_status st, const std::string& msg)
{
    g_err = msg;
    return st;
}

#define HIPCHK(expr)                                                                                      \
    do {                                                                                                  \
        hipError_t e_ = (expr);                                                                           \
        if (e_ != hipSuccess) return fail(TLMPM_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

// Captured pairs of substeps, by the host-side choices they were recorded with
// (label pass, tool contact, rigid contact, slot-table buffer in use).  Every
// per-substep value the kernels need is in device memory (substep index, stamps,
// tools), so a replay equals the launches it was captured from.
struct GraphCache {
    bool on = false;
    hipStream_t cap = nullptr; // capture stream (the caller's may be the null stream)
    std::vector<std::pair<int, hipGraphExec_t>> e;
    ~GraphCache()
    {
        for (auto& x : e) (void)hipGraphExecDestroy(x.second);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

// Kernel timing (diagnostics): pairs of events around launches, per class.  on:
// every launch, each kernel in a launch of its own on the main stream; xfer: only
// the P2G and G2P launches, the launch arrangement left as it is.
struct Timing {
    bool on = false;
    bool xfer = false;
    hipStream_t st = nullptr;
    std::vector<hipEvent_t> pool;
    std::vector<std::pair<int, int>> used; // (class, first event index)
    size_t next = 0;
    ~Timing()
    {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

// A second stream for the launches of a substep that do not depend on the label
// pass or the pair search (rigid contact, slot tables), joined before P2G.  Default
// priority, created on first use.
struct Fork {
    hipStream_t aux = nullptr;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr}; // start, labels done, aux done
    hipError_t init()
    {
        if (aux) return hipSuccess;
        hipError_t e = hipStreamCreateWithFlags(&aux, hipStreamNonBlocking);
        for (int i = 0; i < 3 && e == hipSuccess; i++) e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
        return e;
    }
    ~Fork()
    {
        for (hipEvent_t x : ev)
            if (x) (void)hipEventDestroy(x);
        if (aux) (void)hipStreamDestroy(aux);
    }
};

struct tlmpm_scene {
    SceneK K;
    SceneD D;
    hipStream_t st;
    int max_cuts;
    int n_bricks;
    int cur;       // slot table in use
    int rsb;       // slot table of the pending re-scatter
    bool f_pending; // host copy of the device flag D.ctr[1]
    int in_batch = 0; // member of a live batch: single-scene calls are refused
    int fuse_bricks = 0; // one-stream substeps up to this many active bricks (tuning at creation)
    std::vector<int> active_host;
    Timing prof;
    GraphCache graphs;
    Fork fork;
};

// Brackets one launch with events when timing is on.
struct ProfScope {
    Timing* tm;
    int cls;
    int idx = -1;
    ProfScope(Timing* t, int c) : tm(t), cls(c)
    {
        if (!tm || !(tm->on || (tm->xfer && (c == 0 || c == 1)))) return;
        while (tm->pool.size() < tm->next + 2) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            tm->pool.push_back(e);
        }
        idx = (int)tm->next;
        tm->next += 2;
        (void)hipEventRecord(tm->pool[idx], tm->st);
    }
    ~ProfScope()
    {
        if (idx < 0) return;
        (void)hipEventRecord(tm->pool[idx + 1], tm->st);
        tm->used.push_back({cls, idx});
    }
};

static tlmpm_status timing_read(Timing& tm, int n_classes, double* ms, int64_t* launches);

// the scene needs the general constitutive path of P2G
static int general_path(const SceneK& K) { return K.material == 1 || K.visc > 0.0f || K.ystress > 0.0f; }

static TlLaunch single_launch(const tlmpm_scene* sc)
{
    TlLaunch L;
    memset(&L, 0, sizeof(L));
    L.S = &sc->K;
    L.D = &sc->D;
    L.any_material = sc->K.material_contact;
    L.general = general_path(sc->K);
    L.st = sc->st;
    return L;
}

// ------------------------------------------------------------------- layout
namespace {

struct Layout {
    size_t off = 0;
    size_t take(size_t bytes)
    {
        size_t o = (off + 255) & ~size_t(255);
        off = o + bytes;
        return o;
    }
};

// Launch-shape settings (tlmpm_set_tuning), read when a scene is created or its
// batch footprint is asked for.  Defaults: the measured best on the workloads of
// the benchmark.
static const tlmpm_tuning k_tuning_default = {128, 4096, 512, 4096, 4, 256, 2048, 1};
static tlmpm_tuning g_tuning = k_tuning_default;
static std::mutex g_tuning_mutex;

static tlmpm_tuning tuning_now()
{
    std::lock_guard<std::mutex> lk(g_tuning_mutex);
    return g_tuning;
}

// blocks of the grid-stride pair search of a scene of N particles
int pair_blocks_of(long long N, const tlmpm_tuning& t)
{
    return (int)std::min<long long>(t.pair_cap, std::max<long long>(1, N / t.pair_div));
}

// workgroups for the later same-code rounds of mixed bricks: scenes of split_lo to
// split_hi active bricks only (smaller scenes have few long workgroups to hide,
// larger ones many rounds of workgroups)
int xcap_of(long long n_active, const tlmpm_tuning& t)
{
    return (n_active >= t.split_lo && n_active <= t.split_hi)
               ? (int)std::min<long long>(t.split_cap, n_active / t.split_div)
               : 0;
}

struct Dims {
    long long N;
    int cx, cy, cz, cbx, cby, cbz, nbx, nby, nbz;
    long long NN, n_bricks;
};

Dims dims_of(const tlmpm_scene_desc* d)
{
    Dims g;
    g.N = d->n;
    g.cx = d->cells[0];
    g.cy = d->cells[1];
    g.cz = d->cells[2];
    g.cbx = (g.cx + TL_B - 1) / TL_B;
    g.cby = (g.cy + TL_B - 1) / TL_B;
    g.cbz = (g.cz + TL_B - 1) / TL_B;
    g.nbx = (g.cx >> 2) + 1;
    g.nby = (g.cy >> 2) + 1;
    g.nbz = (g.cz >> 2) + 1;
    g.NN = (long long)g.nbx * g.nby * g.nbz * 64;
    g.n_bricks = (long long)g.cbx * g.cby * g.cbz;
    return g;
}

struct Offsets {
    size_t X, u, v, H, code, code_prev, D, perm, E, m, V0, cell_start, active, cnt0, cnt1, sc0, sc1, p2g, rs, p2g_x,
        rs_x, xp2g, xrs, aabb_x, xlist, xin, xg, hist,
        aabb, wpart, Fdot, Gp, wacc, Jmat, Jrig, brig, bmixed, ccode, ckeys, gmeta, gperm, bround, tools, tinfo, ctr, bact, status, dirty, bdirty, pcell, cand_idx, coff, cmask, cstatic, bcand, hbin, hmax, uanc, uanc_x, uref, bor, umm,
        bcount, bids, crec, htab, hnext, ph_n, ph_q, ph_u,
        qcode, qacc, qrs, qnodes, qround, qmap, total;
    uint32_t hmask;
};

int slot_cap(const tlmpm_scene_desc* d) { return d->slot_capacity > 0 ? d->slot_capacity : 8; }

// reference cell of particle p (FP64), false if it lies outside the grid
bool cell_of(const tlmpm_scene_desc* d, long long p, int c[3])
{
    for (int a = 0; a < 3; a++) {
        double q = ((double)d->X[3 * p + a] - d->origin[a]) / d->dx;
        double fl = std::floor(q);
        if (!(fl >= 0.0) || fl >= (double)d->cells[a]) return false;
        c[a] = (int)fl;
    }
    return true;
}

// Lane map of the quadratic stencil: particle p goes to thread h * 64 + l of its
// brick's workgroup, l its cell slot in the brick (sorted order), h its half pattern
// (bit a set when floor(q_a - 1/2) = floor(q_a), q = (X - origin)/dx: the upper half
// of the cell along axis a, the same FP64 formula as the oracle's stencil); a cell
// with several particles of one pattern gives them successive rounds.  Fills
// lane[p] = h * 64 + l and round[p] when asked; returns the rounds of each brick
// (indexed by brick id, 0 for empty bricks).
std::vector<int> quad_rounds(const tlmpm_scene_desc* d, std::vector<int>* lane, std::vector<int>* round)
{
    Dims g = dims_of(d);
    std::vector<int> rounds((size_t)g.n_bricks, 0);
    std::vector<uint16_t> cnt((size_t)g.n_bricks * 512, 0);
    if (lane) lane->assign((size_t)g.N, -1);
    if (round) round->assign((size_t)g.N, 0);
    for (long long p = 0; p < g.N; p++) {
        int c[3], h = 0;
        if (!cell_of(d, p, c)) continue;
        for (int a = 0; a < 3; a++) {
            const double q = ((double)d->X[3 * p + a] - d->origin[a]) / d->dx;
            if (std::floor(q - 0.5) == std::floor(q)) h |= 1 << a;
        }
        const long long brick = ((long long)(c[2] >> 2) * g.cby + (c[1] >> 2)) * g.cbx + (c[0] >> 2);
        const int lx = c[0] & 3, ly = c[1] & 3, lz = c[2] & 3;
        const int w = (lx & 1) | ((ly & 1) << 1) | ((lz & 1) << 2);
        const int i = (lx >> 1) | ((ly >> 1) << 1) | ((lz >> 1) << 2);
        const int l = w * 8 + i, slot = h * 64 + l;
        const int r = cnt[(size_t)brick * 512 + slot]++;
        rounds[(size_t)brick] = std::max(rounds[(size_t)brick], r + 1);
        if (lane) (*lane)[(size_t)p] = slot;
        if (round) (*round)[(size_t)p] = r;
    }
    return rounds;
}

// number of bricks that hold a particle
long long count_active(const tlmpm_scene_desc* d)
{
    Dims g = dims_of(d);
    std::vector<uint8_t> occ((size_t)g.n_bricks, 0);
    long long n = 0;
    for (long long p = 0; p < g.N; p++) {
        int c[3];
        if (!cell_of(d, p, c)) continue;
        long long b = ((long long)(c[2] >> 2) * g.cby + (c[1] >> 2)) * g.cbx + (c[0] >> 2);
        if (!occ[b]) {
            occ[b] = 1;
            n++;
        }
    }
    return n;
}

Offsets plan(const tlmpm_scene_desc* d, long long n_active)
{
    Dims g = dims_of(d);
    Layout L;
    Offsets o;
    size_t N = (size_t)std::max<long long>(g.N, 1);
    size_t f = sizeof(float);
    o.X = L.take(3 * N * f);
    o.u = L.take(3 * N * f);
    o.v = L.take(3 * N * f);
    o.H = L.take(9 * N * f);
    o.code = L.take(N * 4);
    o.code_prev = L.take(N * 4);
    o.D = L.take(N * f);
    o.perm = L.take(N * 4);
    o.E = d->E ? L.take(N * f) : 0;
    o.m = d->mass ? L.take(N * f) : 0;
    o.V0 = d->vol0 ? L.take(N * f) : 0;
    o.cell_start = L.take(((size_t)g.n_bricks * TL_CELLS + 1) * 4);
    o.active = L.take((size_t)g.n_bricks * 4);
    o.cnt0 = L.take((size_t)g.NN);
    o.cnt1 = L.take((size_t)g.NN);
    const size_t scap = slot_cap(d);
    o.sc0 = L.take((size_t)g.NN * scap * 4);
    o.sc1 = L.take((size_t)g.NN * scap * 4);
    o.p2g = L.take((size_t)n_active * scap * TL_BOXN * 8 * f); // 7 components padded to 8
    o.rs = L.take((size_t)n_active * scap * TL_BOXN * 4 * f);
    o.p2g_x = L.take((size_t)n_active * scap * TL_BOXN * 8 * f);
    o.rs_x = L.take((size_t)n_active * scap * TL_BOXN * 4 * f);
    o.xp2g = L.take((size_t)n_active * 4);
    o.xrs = L.take((size_t)n_active * 4);
    o.aabb_x = L.take((size_t)g.n_bricks * 8 * f);
    o.xlist = L.take((size_t)n_active * 4);
    o.xin = L.take((size_t)n_active * 4);
    o.xg = L.take(4);
    o.bact = L.take((size_t)g.n_bricks * 4);
    o.hist = L.take((size_t)(TL_MAX_TOOLS + 1) * 4 * N * f);
    o.aabb = L.take((size_t)g.n_bricks * 8 * f);
    o.wpart = L.take((size_t)g.n_bricks * TL_MAX_TOOLS * 6 * sizeof(double));
    o.Fdot = d->viscosity > 0.0f ? L.take(9 * N * f) : 0;
    o.Gp = d->yield_stress > 0.0f ? L.take(9 * N * f) : 0;
    o.wacc = L.take(TL_MAX_TOOLS * 6 * sizeof(double));
    o.Jmat = d->material_contact ? L.take(3 * N * f) : 0;
    o.Jrig = L.take(3 * N * f);
    o.brig = L.take((size_t)g.n_bricks * 4);
    o.bmixed = L.take((size_t)g.n_bricks * 4);
    o.ccode = L.take((size_t)g.n_bricks * TL_CELLS * 4);
    o.ckeys = L.take((size_t)g.n_bricks * TL_CELLS * TL_CKEYS * 4);
    o.gmeta = L.take((size_t)n_active * TL_CELLS * TL_GMAX * 4);
    o.gperm = L.take(N * 4);
    o.bround = L.take((size_t)n_active * 4);
    o.tools = L.take(TL_MAX_TOOLS * sizeof(DevTool));
    o.tinfo = L.take(4 * 4);
    o.ctr = L.take(4 * 4);
    o.hmask = 0;
    if (d->material_contact) {
        size_t cells = (size_t)g.n_bricks * TL_CELLS;
        o.cmask = L.take(cells * 4);
        o.cstatic = L.take(cells);
        o.bcand = L.take((size_t)g.n_bricks * 4);
        o.cand_idx = L.take(N * 4);
        o.coff = L.take(((size_t)n_active + 1) * 4);
        o.hbin = L.take(4);
        o.hmax = L.take(TL_HSLOTS * TL_HSTRIDE * 4);
        o.uanc = L.take((size_t)g.n_bricks * 4 * f);
        o.uanc_x = L.take((size_t)g.n_bricks * 4 * f);
        o.uref = L.take((size_t)g.n_bricks * 4 * f);
        o.bor = L.take((size_t)g.n_bricks * 4);
        o.umm = L.take(6 * TL_USLOTS * 4);
        size_t buckets = 4096;
        while (buckets < N / 2) buckets <<= 1;
        o.hmask = (uint32_t)(buckets - 1);
        o.bcount = L.take(2 * buckets * 4);
        o.bids = L.take(buckets * TL_BCAP * 4);
        o.crec = L.take(N * 48);
        o.htab = L.take(buckets * 8);
        o.hnext = L.take(N * 4);
        o.ph_n = L.take(2 * N * 4);
        o.ph_q = L.take(2 * N * TL_PCAP * 4);
        o.ph_u = L.take(2 * N * TL_PCAP * 3 * f);
    }
    o.status = L.take(4);
    o.dirty = L.take(4);
    o.bdirty = L.take((size_t)g.n_bricks * 4);
    o.pcell = L.take(N * 4);
    if (d->stencil == 1) {
        o.qcode = L.take(2 * (size_t)g.NN * scap * 4);
        o.qacc = L.take((size_t)g.NN * scap * 8 * f);
        o.qrs = L.take((size_t)g.NN * scap * 4 * f);
        o.qnodes = L.take((size_t)std::min<long long>(g.NN, n_active * 343) * 4);
        long long total = 0;
        for (int r : quad_rounds(d, nullptr, nullptr)) total += r;
        o.qround = L.take(((size_t)n_active + 1) * 4);
        o.qmap = L.take((size_t)total * TL_WG * 4);
    }
    o.total = L.take(0) + 256;
    return o;
}

tlmpm_status validate(const tlmpm_scene_desc* d)
{
    if (!d) return fail(TLMPM_E_INVALID, "null description");
    if (d->n < 0 || (d->n > 0 && !d->X)) return fail(TLMPM_E_INVALID, "bad particle count or X");
    if (d->n >= (1LL << 31) - 1) return fail(TLMPM_E_INVALID, "more than 2^31-2 particles");
    if (!(d->dx > 0.0) || !(d->dt > 0.0)) return fail(TLMPM_E_INVALID, "dx and dt must be positive");
    for (int a = 0; a < 3; a++)
        if (d->cells[a] <= 0 || d->cells[a] > 1 << 16) return fail(TLMPM_E_INVALID, "cells out of range");
    if (d->max_cuts < 1 || d->max_cuts > 15) return fail(TLMPM_E_INVALID, "max_cuts must be in 1..15");
    if (d->slot_capacity < 0 || d->slot_capacity > TL_SCAP_MAX)
        return fail(TLMPM_E_INVALID, "slot_capacity must be in 0..16 (0: 8)");
    if (d->material != 0 && d->material != 1) return fail(TLMPM_E_INVALID, "material must be 0 or 1");
    if (!(d->viscosity >= 0.0f) || !(d->yield_stress >= 0.0f))
        return fail(TLMPM_E_INVALID, "viscosity and yield_stress must be >= 0");
    if (d->yield_stress > 0.0f && d->material != 1)
        return fail(TLMPM_E_INVALID, "the plasticity projection needs material 1 (fixed-corotated)");
    if (d->stencil != 0 && d->stencil != 1) return fail(TLMPM_E_INVALID, "stencil must be 0 or 1");
    if (d->stencil == 1)
        for (long long p = 0; p < d->n; p++)
            for (int a = 0; a < 3; a++) {
                const double q = ((double)d->X[3 * p + a] - d->origin[a]) / d->dx;
                const double b = std::floor(q - 0.5);
                if (!(b >= 0.0) || b + 2.0 > (double)d->cells[a])
                    return fail(TLMPM_E_INVALID, "particle " + std::to_string(p) +
                                                     ": the quadratic stencil needs half a cell of grid around it");
            }
    if (!(d->nu > -1.0f && d->nu < 0.5f)) return fail(TLMPM_E_INVALID, "nu must be in (-1, 0.5)");
    if (!d->vol0 && !(d->vol0_uniform > 0.0f)) return fail(TLMPM_E_INVALID, "vol0_uniform must be positive");
    if (!d->mass && !(d->mass_uniform > 0.0f)) return fail(TLMPM_E_INVALID, "mass_uniform must be positive");
    if (!d->E && !(d->E_uniform > 0.0f)) return fail(TLMPM_E_INVALID, "E_uniform must be positive");
    Dims g = dims_of(d);
    if (g.n_bricks * TL_CELLS + 1 >= (1LL << 31)) return fail(TLMPM_E_INVALID, "grid too large");
    return TLMPM_OK;
}

bool frame_ok(const tlmpm_blade& b)
{
    auto dot = [](const double* a, const double* c) { return a[0] * c[0] + a[1] * c[1] + a[2] * c[2]; };
    double nn = dot(b.n, b.n), ee = dot(b.e, b.e), dd = dot(b.d, b.d);
    if (std::fabs(std::sqrt(nn) - 1) > 1e-5 || std::fabs(std::sqrt(ee) - 1) > 1e-5 || std::fabs(std::sqrt(dd) - 1) > 1e-5)
        return false;
    if (std::fabs(dot(b.n, b.e)) > 1e-5 || std::fabs(dot(b.n, b.d)) > 1e-5 || std::fabs(dot(b.e, b.d)) > 1e-5)
        return false;
    return b.half_len >= 0 && b.half_width >= 0 && b.b_back >= 0 && b.b_lead >= 0;
}

DevBlade dev_blade(const tlmpm_blade& b)
{
    DevBlade o;
    for (int a = 0; a < 3; a++) {
        o.xe[a] = b.x_e[a];
        o.n[a] = b.n[a];
        o.e[a] = b.e[a];
        o.d[a] = b.d[a];
        o.ve[a] = b.v_e[a];
    }
    o.half_len = b.half_len;
    o.half_width = b.half_width;
    o.b_back = b.b_back;
    o.b_lead = b.b_lead;
    o.cut = b.cut_index;
    o.new_cut = b.new_cut;
    return o;
}

} // namespace

// ------------------------------------------------------------------- ABI
extern "C" const char* tlmpm_last_error(void) { return g_err.c_str(); }

extern "C" tlmpm_status tlmpm_scene_footprint(const tlmpm_scene_desc* desc, size_t* device_bytes)
{
    tlmpm_status s = validate(desc);
    if (s) return s;
    if (!device_bytes) return fail(TLMPM_E_INVALID, "null output");
    *device_bytes = plan(desc, count_active(desc)).total;
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_create_scene(const tlmpm_scene_desc* d, void* ws, size_t bytes, void* hip_stream,
                                           tlmpm_scene** out)
{
    tlmpm_status s = validate(d);
    if (s) return s;
    if (!out) return fail(TLMPM_E_INVALID, "null output");
    *out = nullptr;
    Dims g = dims_of(d);
    const long long N = g.N;

    // reference cell of every particle (FP64, the same formula as the bricks use)
    std::vector<long long> key(N);
    std::vector<int> cnt((size_t)g.n_bricks * TL_CELLS + 1, 0);
    for (long long p = 0; p < N; p++) {
        int c[3];
        if (!cell_of(d, p, c))
            return fail(TLMPM_E_INVALID, "particle " + std::to_string(p) + " lies outside the reference grid");
        long long brick = ((long long)(c[2] >> 2) * g.cby + (c[1] >> 2)) * g.cbx + (c[0] >> 2);
        int lx = c[0] & 3, ly = c[1] & 3, lz = c[2] & 3;
        int w = (lx & 1) | ((ly & 1) << 1) | ((lz & 1) << 2);
        int i = (lx >> 1) | ((ly >> 1) << 1) | ((lz >> 1) << 2);
        key[p] = brick * TL_CELLS + w * 8 + i;
        cnt[key[p] + 1]++;
    }
    for (size_t k = 1; k < cnt.size(); k++) cnt[k] += cnt[k - 1];
    std::vector<int> cell_start(cnt);
    std::vector<int> perm(N);
    {
        std::vector<int> fill(cnt.begin(), cnt.end() - 1);
        for (long long p = 0; p < N; p++) perm[fill[key[p]]++] = (int)p; // stable counting sort
    }
    std::vector<int> active, bact((size_t)g.n_bricks, -1);
    for (long long b = 0; b < g.n_bricks; b++)
        if (cell_start[(b + 1) * TL_CELLS] > cell_start[b * TL_CELLS]) {
            bact[b] = (int)active.size();
            active.push_back((int)b);
        }
    Offsets o = plan(d, (long long)active.size());
    if (!ws || bytes < o.total) return fail(TLMPM_E_NOMEM, "workspace smaller than tlmpm_scene_footprint()");

    tlmpm_scene* sc = new tlmpm_scene();
    sc->st = (hipStream_t)hip_stream;
    sc->prof.st = sc->st;

    sc->max_cuts = d->max_cuts;
    sc->fuse_bricks = tuning_now().one_stream_bricks;
    sc->n_bricks = (int)g.n_bricks;
    sc->cur = 0;
    sc->rsb = 0;
    sc->f_pending = false;
    sc->active_host = active;
    SceneK& K = sc->K;
    memset(&K, 0, sizeof(K));
    K.N = N;
    K.cx = g.cx;
    K.cy = g.cy;
    K.cz = g.cz;
    K.cbx = g.cbx;
    K.cby = g.cby;
    K.cbz = g.cbz;
    K.nbx = g.nbx;
    K.nby = g.nby;
    K.nbz = g.nbz;
    K.NN = g.NN;
    K.ox = d->origin[0];
    K.oy = d->origin[1];
    K.oz = d->origin[2];
    K.dx = d->dx;
    K.inv_dx_d = 1.0 / d->dx;
    K.inv_dx = (float)(1.0 / d->dx);
    K.dt = (float)d->dt;
    K.dt_d = d->dt;
    K.beta = d->flip_beta;
    K.gx = d->gravity[0];
    K.gy = d->gravity[1];
    K.gz = d->gravity[2];
    K.nu = d->nu;
    K.e_uniform = d->E ? 0 : 1;
    K.m_uniform = d->mass ? 0 : 1;
    K.v_uniform = d->vol0 ? 0 : 1;
    K.E0 = d->E_uniform;
    K.m0 = d->mass_uniform;
    K.V0 = d->vol0_uniform;
    K.s_R = d->s_R;
    K.s_n = d->s_n;
    K.gamma_k = d->gamma_k;
    K.gamma_c = d->gamma_c;
    K.mu_s = d->mu_s;
    K.mu_d = d->mu_d;
    K.floor_on = d->floor_on;
    K.floor_z = d->floor_z;
    K.G_c = d->G_c;
    K.zeta = d->zeta;
    K.u_min = d->u_min;
    K.single_field = d->single_field;
    K.material_contact = d->material_contact;
    K.scap = slot_cap(d);
    K.material = d->material;
    K.visc = d->viscosity;
    K.ystress = d->yield_stress;
    const tlmpm_tuning tun = tuning_now();
    K.pair_blocks = pair_blocks_of(N, tun);
    K.stencil = d->stencil;
    K.pair_skip = (d->material_contact && d->stencil == 0 && tun.pair_skip) ? 1 : 0;
    // workgroups for the later rounds of bricks with a mixed cell: a quarter of the
    // bricks, at most 256 (with more mixed bricks no brick is split).  Only scenes of
    // 512 to 4096 active bricks split: their launches are about one round of
    // workgroups on the GPU, so a brick with extra rounds lengthens the whole launch;
    // smaller scenes (the many-scene batches) and larger ones measured slower with the
    // extra launch slots than the rounds cost.
    const size_t na = active.size();
    K.xcap = xcap_of((long long)na, tun);
    float vmax0 = d->vol0_uniform;
    if (d->vol0)
        for (long long p = 0; p < N; p++) vmax0 = std::max(vmax0, d->vol0[p]);
    K.Rmax = 0.5f * d->s_R * std::cbrt(vmax0);

    char* base = (char*)ws;
    SceneD& D = sc->D;
    memset(&D, 0, sizeof(D));
    D.X = (float*)(base + o.X);
    D.u = (float*)(base + o.u);
    D.v = (float*)(base + o.v);
    D.H = (float*)(base + o.H);
    D.code = (uint32_t*)(base + o.code);
    D.code_prev = (uint32_t*)(base + o.code_prev);
    D.D = (float*)(base + o.D);
    D.perm = (int*)(base + o.perm);
    D.E = d->E ? (float*)(base + o.E) : nullptr;
    D.m = d->mass ? (float*)(base + o.m) : nullptr;
    D.V0 = d->vol0 ? (float*)(base + o.V0) : nullptr;
    D.cell_start = (int*)(base + o.cell_start);
    D.active = (int*)(base + o.active);
    D.n_active = (int)active.size();
    D.cnt[0] = (uint8_t*)(base + o.cnt0);
    D.cnt[1] = (uint8_t*)(base + o.cnt1);
    D.scode[0] = (uint32_t*)(base + o.sc0);
    D.scode[1] = (uint32_t*)(base + o.sc1);
    D.p2g = (float*)(base + o.p2g);
    D.rs = (float*)(base + o.rs);
    D.p2g_x = (float*)(base + o.p2g_x);
    D.rs_x = (float*)(base + o.rs_x);
    D.xp2g = (int*)(base + o.xp2g);
    D.xrs = (int*)(base + o.xrs);
    D.aabb_x = (float*)(base + o.aabb_x);
    D.xlist = (int*)(base + o.xlist);
    D.xin = (int*)(base + o.xin);
    D.xg = (int*)(base + o.xg);
    D.hist = (float*)(base + o.hist);
    D.aabb = (float*)(base + o.aabb);
    D.wpart = (double*)(base + o.wpart);
    D.Fdot = o.Fdot ? (float*)(base + o.Fdot) : nullptr;
    D.Gp = o.Gp ? (float*)(base + o.Gp) : nullptr;
    D.wacc = (double*)(base + o.wacc);
    D.Jmat = d->material_contact ? (float*)(base + o.Jmat) : nullptr;
    D.Jrig = (float*)(base + o.Jrig);
    D.brig = (int*)(base + o.brig);
    D.bmixed = (int*)(base + o.bmixed);
    D.ccode = (uint32_t*)(base + o.ccode);
    D.ckeys = (uint32_t*)(base + o.ckeys);
    D.gmeta = (int*)(base + o.gmeta);
    D.gperm = (int*)(base + o.gperm);
    D.bround = (int*)(base + o.bround);
    D.tools = (DevTool*)(base + o.tools);
    D.tinfo = (int*)(base + o.tinfo);
    D.bact = (int*)(base + o.bact);
    D.ctr = (int*)(base + o.ctr);
    if (d->material_contact) {
        D.cmask = (uint32_t*)(base + o.cmask);
        D.cstatic = (uint8_t*)(base + o.cstatic);
        D.bcand = (int*)(base + o.bcand);
        D.cand_idx = (int*)(base + o.cand_idx);
        D.coff = (int*)(base + o.coff);
        D.hbin = (float*)(base + o.hbin);
        D.hmax = (int*)(base + o.hmax);
        D.uanc = (float*)(base + o.uanc);
        D.uanc_x = (float*)(base + o.uanc_x);
        D.uref = (float*)(base + o.uref);
        D.bor = (uint32_t*)(base + o.bor);
        D.umm = (uint32_t*)(base + o.umm);
        D.hmask = o.hmask;
        D.bcount = (int*)(base + o.bcount);
        D.bids = (int*)(base + o.bids);
        D.crec = (float4*)(base + o.crec);
        D.htab = (unsigned long long*)(base + o.htab);
        D.hnext = (int*)(base + o.hnext);
        D.ph_n = (int*)(base + o.ph_n);
        D.ph_q = (int*)(base + o.ph_q);
        D.ph_u = (float*)(base + o.ph_u);
    }
    D.status = (int*)(base + o.status);
    D.dirty = (int*)(base + o.dirty);
    D.bdirty = (int*)(base + o.bdirty);
    D.pcell = (int*)(base + o.pcell);
    std::vector<int> qnodes;
    if (d->stencil == 1) {
        D.qcode = (uint32_t*)(base + o.qcode);
        D.qacc = (float*)(base + o.qacc);
        D.qrs = (float*)(base + o.qrs);
        D.qnodes = (int*)(base + o.qnodes);
        // nodes of the 7x7x7 boxes (from 4 b - 1) of the active bricks, brick-major ids
        std::vector<uint8_t> mark((size_t)g.NN, 0);
        for (int b : active) {
            const int bx = b % g.cbx, by = (b / g.cbx) % g.cby, bz = b / (g.cbx * g.cby);
            for (int z = 0; z < 7; z++)
                for (int y = 0; y < 7; y++)
                    for (int x = 0; x < 7; x++) {
                        const int gx = bx * TL_B - 1 + x, gy = by * TL_B - 1 + y, gz = bz * TL_B - 1 + z;
                        if (gx < 0 || gy < 0 || gz < 0 || gx > g.cx || gy > g.cy || gz > g.cz) continue;
                        const long long nb = ((long long)(gz >> 2) * g.nby + (gy >> 2)) * g.nbx + (gx >> 2);
                        mark[(size_t)((nb << 6) | ((gz & 3) * 16 + (gy & 3) * 4 + (gx & 3)))] = 1;
                    }
        }
        for (long long i = 0; i < g.NN; i++)
            if (mark[(size_t)i]) qnodes.push_back((int)i);
        D.n_qnodes = (int)qnodes.size();
        D.qround = (int*)(base + o.qround);
        D.qmap = (int*)(base + o.qmap);
    }

    // sorted SoA host staging
    std::vector<float> h(3 * (size_t)N);
    auto up3 = [&](float* dst, const float* src) -> hipError_t {
        for (long long q = 0; q < N; q++)
            for (int a = 0; a < 3; a++) h[a * N + q] = src ? src[3 * (size_t)perm[q] + a] : 0.0f;
        hipError_t e = hipMemcpyAsync(dst, h.data(), 3 * N * sizeof(float), hipMemcpyHostToDevice, sc->st);
        if (e == hipSuccess) e = hipStreamSynchronize(sc->st); // h is reused
        return e;
    };
    auto up1 = [&](float* dst, const float* src) -> hipError_t {
        for (long long q = 0; q < N; q++) h[q] = src[perm[q]];
        hipError_t e = hipMemcpyAsync(dst, h.data(), N * sizeof(float), hipMemcpyHostToDevice, sc->st);
        if (e == hipSuccess) e = hipStreamSynchronize(sc->st);
        return e;
    };
    auto bail = [&](hipError_t e, const char* what) {
        delete sc;
        return fail(TLMPM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    hipError_t e;
    if ((e = hipMemsetAsync(ws, 0, o.total - 256, sc->st)) != hipSuccess) return bail(e, "zero workspace");
    if (N > 0) {
        if ((e = up3(D.X, d->X)) != hipSuccess) return bail(e, "upload X");
        if ((e = up3(D.v, d->v0)) != hipSuccess) return bail(e, "upload v0");
        if (d->E && (e = up1(D.E, d->E)) != hipSuccess) return bail(e, "upload E");
        if (d->mass && (e = up1(D.m, d->mass)) != hipSuccess) return bail(e, "upload mass");
        if (d->vol0 && (e = up1(D.V0, d->vol0)) != hipSuccess) return bail(e, "upload vol0");
        if ((e = hipMemcpyAsync(D.perm, perm.data(), N * 4, hipMemcpyHostToDevice, sc->st)) != hipSuccess)
            return bail(e, "upload perm");
        std::vector<int> pc(N);
        for (long long q = 0; q < N; q++) pc[q] = (int)key[perm[q]];
        if ((e = hipMemcpyAsync(D.pcell, pc.data(), N * 4, hipMemcpyHostToDevice, sc->st)) != hipSuccess)
            return bail(e, "upload cells");
        if ((e = hipStreamSynchronize(sc->st)) != hipSuccess) return bail(e, "upload cells");
    }
    if ((e = hipMemcpyAsync(D.cell_start, cell_start.data(), cell_start.size() * 4, hipMemcpyHostToDevice, sc->st)) !=
        hipSuccess)
        return bail(e, "upload cell index");
    if (!active.empty() &&
        (e = hipMemcpyAsync(D.active, active.data(), active.size() * 4, hipMemcpyHostToDevice, sc->st)) != hipSuccess)
        return bail(e, "upload bricks");
    if ((e = hipMemcpyAsync(D.bact, bact.data(), bact.size() * 4, hipMemcpyHostToDevice, sc->st)) != hipSuccess)
        return bail(e, "upload brick index");
    std::vector<int> qround, qmap;
    if (d->stencil == 1) {
        std::vector<int> lane, round;
        const std::vector<int> rounds = quad_rounds(d, &lane, &round);
        qround.assign(active.size() + 1, 0);
        for (size_t b = 0; b < active.size(); b++) qround[b + 1] = qround[b] + rounds[(size_t)active[b]];
        qmap.assign((size_t)qround.back() * TL_WG, -1);
        for (long long q = 0; q < N; q++) { // q: device (sorted) index
            const long long p = perm[(size_t)q];
            const int b = bact[(size_t)(key[(size_t)p] / TL_CELLS)];
            qmap[((size_t)qround[(size_t)b] + round[(size_t)p]) * TL_WG + lane[(size_t)p]] = (int)q;
        }
        if ((e = hipMemcpyAsync(D.qround, qround.data(), qround.size() * 4, hipMemcpyHostToDevice, sc->st)) !=
            hipSuccess)
            return bail(e, "upload lane map");
        if (!qmap.empty() &&
            (e = hipMemcpyAsync(D.qmap, qmap.data(), qmap.size() * 4, hipMemcpyHostToDevice, sc->st)) != hipSuccess)
            return bail(e, "upload lane map");
        if (!qnodes.empty() && (e = hipMemcpyAsync(D.qnodes, qnodes.data(), qnodes.size() * 4, hipMemcpyHostToDevice,
                                                   sc->st)) != hipSuccess)
            return bail(e, "upload stencil nodes");
        if ((e = tl_launch_fill_i32((int*)D.qcode, 2 * g.NN * K.scap, -1, sc->st)) != hipSuccess)
            return bail(e, "init node slots");
        if ((e = hipStreamSynchronize(sc->st)) != hipSuccess) return bail(e, "upload stencil nodes");
    }
    // rigid-contact history stamps start invalid
    if ((e = tl_launch_fill_f32(D.hist, (long long)(TL_MAX_TOOLS + 1) * 4 * N, 0.0f, sc->st)) != hipSuccess)
        return bail(e, "init history");
    // contact-history stamp 1 (stored stamps of 0 read as the previous substep's
    // empty history), no F update pending
    if ((e = tl_launch_fill_i32(D.ctr, 1, 1, sc->st)) != hipSuccess) return bail(e, "counters");
    const TlLaunch L = single_launch(sc);
    if ((e = tl_launch_mixed(&L, 1)) != hipSuccess) return bail(e, "cell summaries");
    if ((e = tl_launch_slots(&L, 0, 0, 1)) != hipSuccess) return bail(e, "slot table");
    if ((e = tl_launch_aabb(&L)) != hipSuccess) return bail(e, "aabb");
    if (d->material_contact) {
        if ((e = tl_launch_cellmask(&L, 1, 1)) != hipSuccess) return bail(e, "cell masks");
        if ((e = tl_launch_cand(&L, 1)) != hipSuccess) return bail(e, "candidates");
    }
    if ((e = hipStreamSynchronize(sc->st)) != hipSuccess) return bail(e, "create");
    *out = sc;
    return TLMPM_OK;
}

static tlmpm_status timing_read(Timing& tm, int n_classes, double* ms, int64_t* launches)
{
    if (n_classes < 0 || n_classes > 6 || (n_classes && (!ms || !launches)))
        return fail(TLMPM_E_INVALID, "bad arguments");
    HIPCHK(hipStreamSynchronize(tm.st));
    for (int c = 0; c < n_classes; c++) {
        ms[c] = 0.0;
        launches[c] = 0;
    }
    for (auto& u : tm.used) {
        float t = 0.0f;
        HIPCHK(hipEventElapsedTime(&t, tm.pool[u.second], tm.pool[u.second + 1]));
        if (u.first < n_classes) {
            ms[u.first] += t;
            launches[u.first] += 1;
        }
    }
    tm.used.clear();
    tm.next = 0;
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_set_tuning(const tlmpm_tuning* t)
{
    tlmpm_tuning v = t ? *t : k_tuning_default;
    if (v.pair_div < 1 || v.pair_cap < 1 || v.split_lo < 0 || v.split_hi < v.split_lo || v.split_div < 1 ||
        v.split_cap < 0 || v.one_stream_bricks < 0 || (v.pair_skip != 0 && v.pair_skip != 1))
        return fail(TLMPM_E_INVALID, "tuning out of range");
    std::lock_guard<std::mutex> lk(g_tuning_mutex);
    g_tuning = v;
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_get_tuning(tlmpm_tuning* t)
{
    if (!t) return fail(TLMPM_E_INVALID, "null output");
    *t = tuning_now();
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_set_graphs(tlmpm_scene* sc, int32_t enable)
{
    if (!sc) return fail(TLMPM_E_INVALID, "null scene");
    sc->graphs.on = enable != 0;
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_profile_enable(tlmpm_scene* sc, int32_t enable)
{
    if (!sc) return fail(TLMPM_E_INVALID, "null scene");
    sc->prof.on = enable == 1;
    sc->prof.xfer = enable == 2;
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_profile_read(tlmpm_scene* sc, int32_t n_classes, double* ms, int64_t* launches)
{
    if (!sc) return fail(TLMPM_E_INVALID, "null scene");
    return timing_read(sc->prof, n_classes, ms, launches);
}

static tlmpm_status refuse_batched(tlmpm_scene* sc);

extern "C" tlmpm_status tlmpm_destroy_scene(tlmpm_scene* sc)
{
    if (tlmpm_status r = refuse_batched(sc)) return r;
    hipError_t e = hipStreamSynchronize(sc->st);
    delete sc;
    if (e != hipSuccess) return fail(TLMPM_E_DEVICE, std::string("destroy: ") + hipGetErrorString(e));
    return TLMPM_OK;
}

// Host side of a run of substeps: the launch context (one scene or a batch) and the
// slot-table bookkeeping shared by every scene it covers.
struct Exec {
    TlLaunch L;
    Timing* prof;      // event timing of the launches, or null
    int cur, rsb;      // slot table in use / of the pending re-scatter
    bool pending;      // some scene has a pending F update
    Fork* fork = nullptr; // second stream, or null (everything on L.st)
    int fuse_bricks = 0;  // single scene: one-stream substeps up to this many active bricks
};

// launches on the second stream (after the main stream's work so far) when there
// is one and timing is off; else on the main stream
struct Side {
    Exec& X;
    TlLaunch La;
    bool par, started = false;
    explicit Side(Exec& x) : X(x), La(x.L)
    {
        par = X.fork && X.fork->aux && !(X.prof && X.prof->on);
        if (par) La.st = X.fork->aux;
    }
    // the second stream waits for what the main stream has queued so far
    hipError_t after_main(int ev)
    {
        if (!par) return hipSuccess;
        started = true;
        hipError_t e = hipEventRecord(X.fork->ev[ev], X.L.st);
        return e != hipSuccess ? e : hipStreamWaitEvent(X.fork->aux, X.fork->ev[ev], 0);
    }
    // the main stream waits for the second stream's work
    hipError_t join()
    {
        if (!started) return hipSuccess;
        started = false;
        hipError_t e = hipEventRecord(X.fork->ev[2], X.fork->aux);
        return e != hipSuccess ? e : hipStreamWaitEvent(X.L.st, X.fork->ev[2], 0);
    }
};

// label pass over the tools flagged TL_TOOL_LABELS (uploaded with their counts),
// then slot-table maintenance and contact candidates of the bricks whose codes
// changed (no host synchronisation).  With a side stream, the slot tables are built
// there, beside the candidates.
static tlmpm_status label_pass(Exec& X, bool reset_D, Side* side = nullptr)
{
    if (reset_D) {
        ProfScope ps(X.prof, 5);
        HIPCHK(tl_launch_resetD(&X.L));
    }
    {
        ProfScope ps(X.prof, 2);
        HIPCHK(tl_launch_labels(&X.L));
    }
    // (cell summaries of the bricks whose codes changed come with the label pass)
    // a pending F update still needs the tables of its re-scatter
    const int dst = (X.pending && X.cur == X.rsb) ? 1 - X.cur : X.cur;
    {
        ProfScope ps(X.prof, 3);
        // the slot tables read the cell summaries and the codes without the
        // candidate bit, which the candidate pass may rewrite meanwhile
        if (side) HIPCHK(side->after_main(1));
        HIPCHK(tl_launch_slots(side ? &side->La : &X.L, dst, X.cur, 0));
    }
    X.cur = dst;
    if (X.L.any_material) { // cell code masks come with the cell summaries (k_mixed)
        ProfScope ps(X.prof, 4);
        HIPCHK(tl_launch_cand(&X.L, 0));
    }
    return TLMPM_OK;
}

struct CallFlags {
    bool any_labels = false, any_new = false, any_contact_tool = false, any_rigid = false;
};

// one substep of the whole path.  With material contact and a side stream, the
// launches that do not depend on the pair search run beside it: rigid contact
// (reads only the last substep's motion, the tools and the cutting progress, reset
// first when a cut starts) from the start of the substep, the slot tables after the
// label pass; P2G waits for them.
// one substep with the quadratic stencil: labels and contact as in the trilinear
// path, then the transfers of tlmpm_quad.hip with the node tables of parity X.cur
// (flipped every substep); the F update completes inside the substep.
// Single scenes of at most X.fuse_bricks active bricks (tlmpm_tuning.one_stream_bricks
// when the scene was created) run a substep with a label pass on one stream (see
// fused_label_substep).
static bool one_stream(const Exec& X, const CallFlags& f)
{
    return f.any_labels && X.L.S && X.L.D->n_active <= X.fuse_bricks && !(X.prof && X.prof->on);
}

static tlmpm_status one_substep_quad(Exec& X, const CallFlags& f, bool first)
{
    const bool fused = one_stream(X, f); // label pass and rigid contact in one launch
    Side side(X);
    side.par = side.par && X.L.any_material && !fused;
    if (f.any_labels && f.any_new && first) {
        ProfScope ps(X.prof, 5);
        HIPCHK(tl_launch_resetD(&X.L));
    }
    if (fused) {
        HIPCHK(f.any_rigid ? tl_launch_labels_rigid(&X.L) : tl_launch_labels(&X.L));
    } else {
        if (f.any_rigid && side.par) {
            HIPCHK(side.after_main(0));
            HIPCHK(tl_launch_rigid(&side.La));
        }
        if (f.any_labels) {
            ProfScope ps(X.prof, 2);
            HIPCHK(tl_launch_labels(&X.L));
        }
    }
    {
        ProfScope ps(X.prof, 3);
        HIPCHK(tl_launch_quad(&X.L, X.cur, 0));
    }
    if (X.L.any_material) {
        ProfScope ps(X.prof, 4);
        if (f.any_labels) HIPCHK(tl_launch_cand(&X.L, 0));
        HIPCHK(tl_launch_contact(&X.L));
    }
    if (f.any_rigid && !side.par && !fused) {
        ProfScope ps(X.prof, 5);
        HIPCHK(tl_launch_rigid(&X.L));
    }
    HIPCHK(side.join());
    const int cls[6] = {3, 0, 5, 1, 5, 5};
    for (int stage = 1; stage < 6; stage++) {
        ProfScope ps(X.prof, cls[stage]);
        HIPCHK(tl_launch_quad(&X.L, X.cur, stage));
    }
    X.cur = 1 - X.cur;
    return TLMPM_OK;
}

// A substep of one scene with a label pass, untimed: one stream, with the label pass
// and rigid contact in one launch and the slot tables in the launch of the pair
// search (each pair touches disjoint arrays), instead of the second stream, whose
// fork and join events cost more than the launches they overlap; the binning blocks
// sum the candidate offsets themselves (no scan launch).  Only scenes of at
// most one_stream_bricks active bricks: there the two launches of a pair fit the chip
// side by side; a large scene (27k bricks) measured slower fused (labels and rigid
// contact 0.22 ms against 0.06 ms with rigid contact beside it), and batches keep the
// second stream as well.
static tlmpm_status fused_label_substep(Exec& X, const CallFlags& f)
{
    HIPCHK(f.any_rigid ? tl_launch_labels_rigid(&X.L) : tl_launch_labels(&X.L));
    // a pending F update still needs the tables of its re-scatter
    const int dst = (X.pending && X.cur == X.rsb) ? 1 - X.cur : X.cur;
    if (X.L.any_material) {
        HIPCHK(tl_launch_cand_contact_slots(&X.L, dst, X.cur));
    } else {
        HIPCHK(tl_launch_slots(&X.L, dst, X.cur, 0));
    }
    X.cur = dst;
    return TLMPM_OK;
}

static tlmpm_status one_substep(Exec& X, const CallFlags& f, bool first)
{
    if (X.L.S && X.L.S->stencil == 1) return one_substep_quad(X, f, first);
    const bool fused = one_stream(X, f);
    Side side(X);
    side.par = side.par && X.L.any_material && !fused;
    const bool reset_D = f.any_labels && f.any_new && first;
    if (reset_D) {
        ProfScope ps(X.prof, 5);
        HIPCHK(tl_launch_resetD(&X.L));
    }
    if (fused) {
        tlmpm_status s = fused_label_substep(X, f);
        if (s) return s;
    } else {
        if (f.any_rigid && side.par) {
            HIPCHK(side.after_main(0));
            HIPCHK(tl_launch_rigid(&side.La));
        }
        if (f.any_labels) {
            tlmpm_status s = label_pass(X, false, side.par ? &side : nullptr);
            if (s) return s;
        }
        if (X.L.any_material) {
            ProfScope ps(X.prof, 4);
            HIPCHK(tl_launch_contact(&X.L));
        }
        if (f.any_rigid && !side.par) {
            ProfScope ps(X.prof, 5);
            HIPCHK(tl_launch_rigid(&X.L));
        }
        HIPCHK(side.join());
    }
    {
        ProfScope ps(X.prof, 0);
        HIPCHK(tl_launch_p2g(&X.L, 1, X.cur != X.rsb ? 1 : 0, X.cur, X.rsb));
    }
    {
        ProfScope ps(X.prof, 1);
        HIPCHK(tl_launch_g2p(&X.L, X.cur));
    }
    X.pending = true;
    X.rsb = X.cur;
    return TLMPM_OK;
}

static tlmpm_status pair_graph(Exec& X, const CallFlags& f, GraphCache& gc, hipGraphExec_t* out)
{
    const int key = (f.any_labels ? 1 : 0) | (f.any_contact_tool ? 2 : 0) | (f.any_rigid ? 4 : 0) | (X.cur << 3);
    for (auto& x : gc.e)
        if (x.first == key) {
            *out = x.second;
            return TLMPM_OK;
        }
    if (!gc.cap) HIPCHK(hipStreamCreateWithFlags(&gc.cap, hipStreamNonBlocking));
    // record the launches on the capture stream (nothing runs); replays go to the
    // scene's stream, ordered after the work queued there
    Exec Y = X;
    Y.prof = nullptr;
    Y.L.st = gc.cap;
    HIPCHK(hipStreamBeginCapture(Y.L.st, hipStreamCaptureModeThreadLocal));
    tlmpm_status s = one_substep(Y, f, false);
    if (!s) s = one_substep(Y, f, false);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(Y.L.st, &g);
    if (s) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess) return fail(TLMPM_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    if (Y.cur != X.cur || Y.rsb != X.rsb) {
        (void)hipGraphDestroy(g);
        return fail(TLMPM_E_DEVICE, "graph capture: slot-table state not periodic");
    }
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiateWithFlags(&ex, g, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(TLMPM_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    gc.e.push_back({key, ex});
    *out = ex;
    return TLMPM_OK;
}

// n_substeps substeps of the whole path.  With graphs on (and no kernel timing),
// the substeps after the first run as replays of a captured pair of substeps.
static tlmpm_status run_substeps(Exec& X, int n_substeps, const CallFlags& f, GraphCache* gc = nullptr)
{
    HIPCHK(tl_launch_call_start(&X.L)); // substep index 0, interval wrench cleared
    int j = 0;
    if (n_substeps > 0) {
        tlmpm_status s = one_substep(X, f, true);
        if (s) return s;
        j = 1;
    }
    if (gc && gc->on && !(X.prof && X.prof->on) && X.pending && X.cur == X.rsb) {
        for (; j + 2 <= n_substeps; j += 2) {
            hipGraphExec_t ex = nullptr;
            tlmpm_status s = pair_graph(X, f, *gc, &ex);
            if (s) return s;
            HIPCHK(hipGraphLaunch(ex, X.L.st));
        }
    }
    for (; j < n_substeps; j++) {
        tlmpm_status s = one_substep(X, f, false);
        if (s) return s;
    }
    if (f.any_contact_tool) { // the call's wrench from the per-brick sums
        ProfScope ps(X.prof, 5);
        HIPCHK(tl_launch_wrench(&X.L));
    }
    return TLMPM_OK;
}

static Exec single_exec(tlmpm_scene* sc)
{
    Exec X;
    X.L = single_launch(sc);
    X.prof = &sc->prof;
    X.fork = &sc->fork;
    X.cur = sc->cur;
    X.rsb = sc->rsb;
    X.pending = sc->f_pending;
    X.fuse_bricks = sc->fuse_bricks;
    return X;
}

static void single_done(tlmpm_scene* sc, const Exec& X)
{
    sc->cur = X.cur;
    sc->rsb = X.rsb;
    sc->f_pending = X.pending;
}

static tlmpm_status upload_tools(tlmpm_scene* sc, const DevTool* t, int n, const int tinfo[4])
{
    if (n > 0) HIPCHK(hipMemcpyAsync(sc->D.tools, t, n * sizeof(DevTool), hipMemcpyHostToDevice, sc->st));
    HIPCHK(hipMemcpyAsync(sc->D.tinfo, tinfo, 4 * sizeof(int), hipMemcpyHostToDevice, sc->st));
    return TLMPM_OK;
}

static tlmpm_status refuse_batched(tlmpm_scene* sc)
{
    if (!sc) return fail(TLMPM_E_INVALID, "null scene");
    if (sc->in_batch) return fail(TLMPM_E_INVALID, "scene belongs to a live batch (destroy the batch first)");
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_assign_labels(tlmpm_scene* sc, const tlmpm_blade* blades, int32_t n_blades)
{
    if (tlmpm_status r = refuse_batched(sc)) return r;
    if ((n_blades > 0 && !blades) || n_blades < 0 || n_blades > TL_MAX_TOOLS)
        return fail(TLMPM_E_INVALID, "bad arguments (at most 4 blades)");
    DevTool t[TL_MAX_TOOLS];
    memset(t, 0, sizeof(t));
    bool any_new = false;
    for (int b = 0; b < n_blades; b++) {
        const tlmpm_blade& B = blades[b];
        if (B.cut_index < 0 || B.cut_index >= sc->max_cuts) return fail(TLMPM_E_INVALID, "cut_index out of range");
        if (!frame_ok(B)) return fail(TLMPM_E_INVALID, "blade frame (n, e, d) must be orthonormal");
        t[b].b = dev_blade(B);
        t[b].flags = TL_TOOL_LABELS;
        t[b].slot = 1 + b;
        any_new |= B.new_cut != 0;
    }
    if (n_blades == 0) return TLMPM_OK;
    const int tinfo[4] = {n_blades, 0, any_new ? 1 : 0, 0};
    tlmpm_status s = upload_tools(sc, t, n_blades, tinfo);
    if (s) return s;
    Exec X = single_exec(sc);
    X.fork = nullptr;
    s = label_pass(X, any_new);
    single_done(sc, X);
    return s;
}

// applies a pending F update on its own (before host access to the state)
static tlmpm_status flush_F(tlmpm_scene* sc)
{
    if (!sc->f_pending) return TLMPM_OK;
    const TlLaunch L = single_launch(sc);
    HIPCHK(tl_launch_p2g(&L, 0, sc->cur != sc->rsb ? 1 : 0, sc->cur, sc->rsb));
    HIPCHK(tl_launch_fill_i32(sc->D.ctr + 1, 1, 0, sc->st));
    sc->f_pending = false;
    return TLMPM_OK;
}

// checks the tools of one scene and converts them to the device form; returns the
// per-call flags and the device tool info (count, any contact, new cut)
static tlmpm_status convert_tools(const tlmpm_scene* sc, const tlmpm_tool* tools, int n_tools, DevTool* dtl,
                                  int tinfo[4], CallFlags& f)
{
    memset(dtl, 0, TL_MAX_TOOLS * sizeof(DevTool));
    bool any_contact_tool = false, any_labels = false, any_new = false;
    for (int t = 0; t < n_tools; t++) {
        const tlmpm_tool& T = tools[t];
        const tlmpm_blade& B = T.blade;
        if (!frame_ok(B)) return fail(TLMPM_E_INVALID, "tool frame (n, e, d) must be orthonormal");
        if ((T.flags & TLMPM_TOOL_LABELS) && (B.cut_index < 0 || B.cut_index >= sc->max_cuts))
            return fail(TLMPM_E_INVALID, "cut_index out of range");
        if ((T.flags & TLMPM_TOOL_ADVANCE) && (T.omega_B[0] != 0 || T.omega_B[1] != 0 || T.omega_B[2] != 0))
            return fail(TLMPM_E_INVALID, "TLMPM_TOOL_ADVANCE supports translating tools only");
        DevTool& o = dtl[t];
        o.b = dev_blade(B);
        for (int a = 0; a < 3; a++) {
            o.xB[a] = T.x_B[a];
            o.vB[a] = T.v_B[a];
            o.wB[a] = (float)T.omega_B[a];
        }
        o.invm = (float)T.w_B;
        o.imass = (float)T.inv_mass;
        for (int a = 0; a < 9; a++) o.iinv[a] = (float)T.inv_inertia[a];
        o.flags = T.flags;
        o.slot = 1 + t;
        any_contact_tool |= (T.flags & TLMPM_TOOL_CONTACT) != 0;
        any_labels |= (T.flags & TLMPM_TOOL_LABELS) != 0;
        any_new |= (T.flags & TLMPM_TOOL_LABELS) && B.new_cut;
    }
    tinfo[0] = n_tools;
    tinfo[1] = any_contact_tool ? 1 : 0;
    tinfo[2] = any_new ? 1 : 0;
    tinfo[3] = 0;
    f.any_labels |= any_labels;
    f.any_new |= any_new;
    f.any_contact_tool |= any_contact_tool;
    f.any_rigid |= any_contact_tool || sc->K.floor_on;
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_step(tlmpm_scene* sc, const tlmpm_tool* tools, int32_t n_tools, int32_t n_substeps,
                                   double* wrench)
{
    if (tlmpm_status r = refuse_batched(sc)) return r;
    if (n_tools < 0 || n_tools > TL_MAX_TOOLS || (n_tools > 0 && !tools) || n_substeps < 0)
        return fail(TLMPM_E_INVALID, "bad arguments (at most 4 tools)");
    DevTool dtl[TL_MAX_TOOLS];
    int tinfo[4];
    CallFlags f;
    tlmpm_status s = convert_tools(sc, tools, n_tools, dtl, tinfo, f);
    if (s) return s;
    s = upload_tools(sc, dtl, n_tools, tinfo);
    if (s) return s;
    HIPCHK(sc->fork.init());
    Exec X = single_exec(sc);
    s = run_substeps(X, n_substeps, f, &sc->graphs);
    single_done(sc, X);
    if (s) return s;
    if (wrench && n_tools > 0) {
        double acc[TL_MAX_TOOLS * 6];
        if (f.any_contact_tool) {
            HIPCHK(hipMemcpyAsync(acc, sc->D.wacc, n_tools * 6 * sizeof(double), hipMemcpyDeviceToHost, sc->st));
            HIPCHK(hipStreamSynchronize(sc->st));
        } else {
            for (int q = 0; q < n_tools * 6; q++) acc[q] = 0.0;
        }
        double inv = n_substeps > 0 ? 1.0 / n_substeps : 0.0;
        for (int q = 0; q < n_tools * 6; q++) wrench[q] = acc[q] * inv;
    }
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_get_status(tlmpm_scene* sc, int32_t* status)
{
    if (tlmpm_status r = refuse_batched(sc)) return r;
    if (!status) return fail(TLMPM_E_INVALID, "bad arguments");
    int st = 0;
    HIPCHK(hipMemcpyAsync(&st, sc->D.status, 4, hipMemcpyDeviceToHost, sc->st));
    HIPCHK(hipStreamSynchronize(sc->st));
    *status = 0;
    if (st & TL_ST_NONFINITE) *status = TLMPM_E_NONFINITE;
    if (st & (TL_ST_SLOT | TL_ST_BOX | TL_ST_LOOKUP | TL_ST_CONTACT)) *status = TLMPM_E_SLOT_OVERFLOW;
    if (st) g_err = "device status bits " + std::to_string(st);
    return TLMPM_OK;
}

static uint64_t code_to_ternary(uint32_t c, int K)
{
    uint64_t v = 0, w = 1;
    for (int k = 0; k < K; k++) {
        int dg = (c >> k) & 1 ? 1 : ((c >> (15 + k)) & 1 ? 2 : 0);
        v += (uint64_t)dg * w;
        w *= 3;
    }
    return v;
}

extern "C" tlmpm_status tlmpm_read_state(tlmpm_scene* sc, uint32_t mask, void* const* out)
{
    if (tlmpm_status r = refuse_batched(sc)) return r;
    if (mask && !out) return fail(TLMPM_E_INVALID, "bad arguments");
    tlmpm_status s = flush_F(sc);
    if (s) return s;
    const long long N = sc->K.N;
    SceneD& D = sc->D;
    std::vector<int> perm(N);
    if (N) HIPCHK(hipMemcpyAsync(perm.data(), D.perm, N * 4, hipMemcpyDeviceToHost, sc->st));
    std::vector<float> buf;
    std::vector<uint32_t> cb;
    HIPCHK(hipStreamSynchronize(sc->st));
    int slot = 0;
    for (uint32_t bit = 1; bit <= TLMPM_FIELD_H; bit <<= 1) {
        if (!(mask & bit)) continue;
        void* dst = out[slot++];
        if (!dst) return fail(TLMPM_E_INVALID, "null output buffer");
        if (bit == TLMPM_FIELD_X || bit == TLMPM_FIELD_U || bit == TLMPM_FIELD_V || bit == TLMPM_FIELD_F ||
            bit == TLMPM_FIELD_D || bit == TLMPM_FIELD_H) {
            int comps = (bit == TLMPM_FIELD_F || bit == TLMPM_FIELD_H) ? 9 : (bit == TLMPM_FIELD_D ? 1 : 3);
            const float* src = bit == TLMPM_FIELD_X ? D.X
                               : bit == TLMPM_FIELD_U ? D.u
                               : bit == TLMPM_FIELD_V ? D.v
                               : (bit == TLMPM_FIELD_F || bit == TLMPM_FIELD_H) ? D.H
                                                                                : D.D;
            buf.resize((size_t)comps * N);
            if (N) HIPCHK(hipMemcpyAsync(buf.data(), src, (size_t)comps * N * 4, hipMemcpyDeviceToHost, sc->st));
            HIPCHK(hipStreamSynchronize(sc->st));
            float* o = (float*)dst;
            for (long long q = 0; q < N; q++)
                for (int a = 0; a < comps; a++) {
                    float val = buf[(size_t)a * N + q];
                    if (bit == TLMPM_FIELD_F && (a == 0 || a == 4 || a == 8)) val += 1.0f;
                    o[(size_t)perm[q] * comps + a] = val;
                }
        } else {
            cb.resize(N);
            if (N) HIPCHK(hipMemcpyAsync(cb.data(), D.code, N * 4, hipMemcpyDeviceToHost, sc->st));
            HIPCHK(hipStreamSynchronize(sc->st));
            for (long long q = 0; q < N; q++) {
                uint32_t c = cb[q];
                if (bit == TLMPM_FIELD_CODE) {
                    ((uint64_t*)dst)[perm[q]] = code_to_ternary(c, sc->max_cuts);
                } else {
                    uint8_t* o = (uint8_t*)dst + (size_t)perm[q] * sc->max_cuts;
                    for (int k = 0; k < sc->max_cuts; k++)
                        o[k] = (c >> k) & 1 ? 1 : ((c >> (15 + k)) & 1 ? 2 : 0);
                }
            }
        }
    }
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_write_state(tlmpm_scene* sc, uint32_t mask, const void* const* in)
{
    if (tlmpm_status r = refuse_batched(sc)) return r;
    if (mask && !in) return fail(TLMPM_E_INVALID, "bad arguments");
    if (mask & (TLMPM_FIELD_X | TLMPM_FIELD_CODE)) return fail(TLMPM_E_INVALID, "X and CODE are not writable");
    if ((mask & TLMPM_FIELD_F) && (mask & TLMPM_FIELD_H)) return fail(TLMPM_E_INVALID, "write F or H, not both");
    tlmpm_status s = flush_F(sc);
    if (s) return s;
    const long long N = sc->K.N;
    SceneD& D = sc->D;
    std::vector<int> perm(N);
    if (N) HIPCHK(hipMemcpyAsync(perm.data(), D.perm, N * 4, hipMemcpyDeviceToHost, sc->st));
    HIPCHK(hipStreamSynchronize(sc->st));
    std::vector<float> buf;
    int slot = 0;
    bool codes_changed = false;
    for (uint32_t bit = 1; bit <= TLMPM_FIELD_H; bit <<= 1) {
        if (!(mask & bit)) continue;
        const void* src = in[slot++];
        if (!src) return fail(TLMPM_E_INVALID, "null input buffer");
        if (bit == TLMPM_FIELD_DIGITS) {
            std::vector<uint32_t> cb(N);
            const uint8_t* dg = (const uint8_t*)src;
            for (long long q = 0; q < N; q++) {
                uint32_t c = 0;
                for (int k = 0; k < sc->max_cuts; k++) {
                    uint8_t v = dg[(size_t)perm[q] * sc->max_cuts + k];
                    if (v > 2) return fail(TLMPM_E_INVALID, "digits must be 0, 1 or 2");
                    if (v == 1) c |= 1u << k;
                    if (v == 2) c |= 1u << (15 + k);
                }
                cb[q] = c;
            }
            if (N) HIPCHK(hipMemcpyAsync(D.code, cb.data(), N * 4, hipMemcpyHostToDevice, sc->st));
            HIPCHK(hipStreamSynchronize(sc->st));
            codes_changed = true;
            continue;
        }
        int comps = (bit == TLMPM_FIELD_F || bit == TLMPM_FIELD_H) ? 9 : (bit == TLMPM_FIELD_D ? 1 : 3);
        float* dstp = bit == TLMPM_FIELD_U   ? D.u
                      : bit == TLMPM_FIELD_V ? D.v
                      : (bit == TLMPM_FIELD_F || bit == TLMPM_FIELD_H) ? D.H
                                                                       : D.D;
        buf.resize((size_t)comps * N);
        const float* f = (const float*)src;
        for (long long q = 0; q < N; q++)
            for (int a = 0; a < comps; a++) {
                float val = f[(size_t)perm[q] * comps + a];
                if (bit == TLMPM_FIELD_F && (a == 0 || a == 4 || a == 8)) val -= 1.0f;
                buf[(size_t)a * N + q] = val;
            }
        if (N) HIPCHK(hipMemcpyAsync(dstp, buf.data(), (size_t)comps * N * 4, hipMemcpyHostToDevice, sc->st));
        HIPCHK(hipStreamSynchronize(sc->st));
    }
    const TlLaunch L = single_launch(sc);
    if (codes_changed) {
        // the list of bricks with a mixed cell is rebuilt with the summaries
        HIPCHK(tl_launch_fill_i32(sc->D.xin, sc->D.n_active, 0, sc->st));
        HIPCHK(tl_launch_fill_i32(sc->D.ctr + 3, 1, 0, sc->st));
        HIPCHK(tl_launch_mixed(&L, 1));
        HIPCHK(tl_launch_slots(&L, sc->cur, sc->cur, 1));
        sc->rsb = sc->cur;
        if (sc->K.material_contact) HIPCHK(tl_launch_cand(&L, 1));
    }
    // speed bounds of the new velocities replace those gathered by the last G2P
    if (sc->K.material_contact) HIPCHK(tl_launch_fill_i32(sc->D.hmax, TL_HSLOTS * TL_HSTRIDE, 0, sc->st));
    if (sc->K.pair_skip) HIPCHK(tl_launch_fill_i32((int*)sc->D.umm, 6 * TL_USLOTS, 0, sc->st));
    HIPCHK(tl_launch_aabb(&L));
    HIPCHK(hipStreamSynchronize(sc->st));
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_slot_stats(tlmpm_scene* sc, int64_t* total_slots, int32_t* max_per_node)
{
    if (tlmpm_status r = refuse_batched(sc)) return r;
    std::vector<uint8_t> c(sc->K.NN);
    HIPCHK(hipMemcpyAsync(c.data(), sc->D.cnt[sc->cur], sc->K.NN, hipMemcpyDeviceToHost, sc->st));
    HIPCHK(hipStreamSynchronize(sc->st));
    int64_t tot = 0;
    int mx = 0;
    for (uint8_t v : c) {
        tot += v;
        mx = std::max(mx, (int)v);
    }
    if (total_slots) *total_slots = tot;
    if (max_per_node) *max_per_node = mx;
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_slot_histogram(tlmpm_scene* sc, int64_t hist[TL_SCAP_MAX + 1])
{
    if (!hist) return fail(TLMPM_E_INVALID, "null output");
    if (tlmpm_status r = refuse_batched(sc)) return r;
    std::vector<uint8_t> c(sc->K.NN);
    HIPCHK(hipMemcpyAsync(c.data(), sc->D.cnt[sc->cur], sc->K.NN, hipMemcpyDeviceToHost, sc->st));
    HIPCHK(hipStreamSynchronize(sc->st));
    for (int i = 0; i <= TL_SCAP_MAX; i++) hist[i] = 0;
    for (uint8_t v : c) hist[std::min<int>(v, TL_SCAP_MAX)]++;
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_contact_stats(tlmpm_scene* sc, double out[8])
{
    if (!out) return fail(TLMPM_E_INVALID, "null output");
    if (tlmpm_status r = refuse_batched(sc)) return r;
    for (int i = 0; i < 8; i++) out[i] = 0.0;
    if (!sc->K.material_contact) return TLMPM_OK;
    const size_t nb = (size_t)sc->D.hmask + 1;
    std::vector<int> cnt(nb);
    int total = 0, stamp = 0;
    float hb = 0.0f;
    HIPCHK(hipMemcpyAsync(&stamp, sc->D.ctr, 4, hipMemcpyDeviceToHost, sc->st));
    HIPCHK(hipStreamSynchronize(sc->st));
    // counts of the last substep: the buffer of its stamp (the current one minus one)
    const int* src = sc->D.bcount + (size_t)((stamp - 1) & 1) * nb;
    HIPCHK(hipMemcpyAsync(cnt.data(), src, nb * 4, hipMemcpyDeviceToHost, sc->st));
    HIPCHK(hipMemcpyAsync(&total, sc->D.coff + sc->D.n_active, 4, hipMemcpyDeviceToHost, sc->st));
    HIPCHK(hipMemcpyAsync(&hb, sc->D.hbin, 4, hipMemcpyDeviceToHost, sc->st));
    HIPCHK(hipStreamSynchronize(sc->st));
    long long used = 0, over = 0;
    int mx = 0;
    for (int c : cnt) {
        used += c > 0;
        over += c > TL_BCAP;
        mx = std::max(mx, c);
    }
    out[0] = total;
    out[1] = (double)nb;
    out[2] = (double)used;
    out[3] = (double)over;
    out[4] = mx;
    out[5] = hb;
    // pairs in contact: every contact is kept in both partners' spring lists of
    // the substep's stamp (at most TL_PCAP per particle)
    const long long N = sc->K.N;
    std::vector<int> hdr((size_t)N);
    HIPCHK(hipMemcpyAsync(hdr.data(), sc->D.ph_n + (size_t)((stamp - 1) & 1) * N, (size_t)N * 4,
                          hipMemcpyDeviceToHost, sc->st));
    HIPCHK(hipStreamSynchronize(sc->st));
    long long ends = 0;
    for (int h : hdr)
        if ((h >> 8) == stamp - 1) ends += h & 0xFF;
    out[6] = 0.5 * (double)ends;
    // candidates the binning marked as without a possible partner (first vector of
    // each record: the flag beside the cell's z); the whole records are copied
    if (total > 0) {
        std::vector<float4> rec((size_t)total * 3);
        HIPCHK(hipMemcpyAsync(rec.data(), sc->D.crec, rec.size() * sizeof(float4), hipMemcpyDeviceToHost, sc->st));
        HIPCHK(hipStreamSynchronize(sc->st));
        long long skipped = 0;
        for (size_t g = 0; g < (size_t)total; g++) {
            int w;
            std::memcpy(&w, &rec[3 * g].w, 4);
            skipped += (w >> 30) & 1;
        }
        out[7] = (double)skipped;
    }
    return TLMPM_OK;
}

// ------------------------------------------------------------- rigid tool body
namespace {
// rotation matrix (row major) of the unit quaternion (w, x, y, z)
void quat_rot(const double q[4], double R[9])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z);
    R[1] = 2 * (x * y - w * z);
    R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);
    R[4] = 1 - 2 * (x * x + z * z);
    R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);
    R[7] = 2 * (y * z + w * x);
    R[8] = 1 - 2 * (x * x + y * y);
}

void mat_vec(const double M[9], const double a[3], double out[3])
{
    for (int i = 0; i < 3; i++) out[i] = M[3 * i] * a[0] + M[3 * i + 1] * a[1] + M[3 * i + 2] * a[2];
}

void mat_tvec(const double M[9], const double a[3], double out[3]) // M^T a
{
    for (int i = 0; i < 3; i++) out[i] = M[i] * a[0] + M[3 + i] * a[1] + M[6 + i] * a[2];
}

void cross(const double a[3], const double b[3], double out[3])
{
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

bool body_ok(const tlmpm_rigid_body* b)
{
    if (!b || !(b->mass > 0.0) || !std::isfinite(b->mass)) return false;
    double qq = 0.0;
    for (int i = 0; i < 4; i++) qq += b->q[i] * b->q[i];
    if (!(qq > 0.0) || !std::isfinite(qq)) return false;
    for (int i = 0; i < 3; i++)
        if (!(b->inertia[i] > 0.0) || !std::isfinite(b->inertia[i])) return false;
    return true;
}
} // namespace

extern "C" tlmpm_status tlmpm_rigid_step(tlmpm_rigid_body* body, const double wrench[6], const double gravity[3], double h)
{
    if (!body || !wrench || !gravity || !(h > 0.0)) return fail(TLMPM_E_INVALID, "bad arguments");
    if (!body_ok(body)) return fail(TLMPM_E_INVALID, "body needs mass > 0, moments > 0 and a nonzero quaternion");
    tlmpm_rigid_body b = *body;
    double R[9];
    quat_rot(b.q, R);
    // linear momentum
    for (int a = 0; a < 3; a++) b.v[a] += h * (wrench[a] / b.mass + gravity[a]);
    // Euler's equations in body axes (explicit gyroscopic term)
    double wb[3], tb[3], Iw[3], g[3];
    mat_tvec(R, b.omega, wb);
    mat_tvec(R, wrench + 3, tb);
    for (int a = 0; a < 3; a++) Iw[a] = b.inertia[a] * wb[a];
    cross(wb, Iw, g);
    for (int a = 0; a < 3; a++) wb[a] += h * (tb[a] - g[a]) / b.inertia[a];
    mat_vec(R, wb, b.omega);
    // position and orientation from the new velocities
    for (int a = 0; a < 3; a++) b.x[a] += h * b.v[a];
    const double w = b.q[0], x = b.q[1], y = b.q[2], z = b.q[3];
    const double* o = b.omega;
    double dq[4] = {-(o[0] * x + o[1] * y + o[2] * z), o[0] * w + o[1] * z - o[2] * y, o[1] * w + o[2] * x - o[0] * z,
                    o[2] * w + o[0] * y - o[1] * x}; // (0, omega) q
    double nq = 0.0;
    for (int i = 0; i < 4; i++) {
        b.q[i] += 0.5 * h * dq[i];
        nq += b.q[i] * b.q[i];
    }
    nq = std::sqrt(nq);
    for (int i = 0; i < 4; i++) b.q[i] /= nq;
    bool fin = true;
    for (int a = 0; a < 3; a++) fin = fin && std::isfinite(b.x[a]) && std::isfinite(b.v[a]) && std::isfinite(b.omega[a]);
    for (int i = 0; i < 4; i++) fin = fin && std::isfinite(b.q[i]);
    if (!fin) return fail(TLMPM_E_INVALID, "rigid step not finite");
    *body = b;
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_rigid_tool(const tlmpm_rigid_body* body, const tlmpm_blade* bb, uint32_t flags,
                                         tlmpm_tool* out)
{
    if (!bb || !out) return fail(TLMPM_E_INVALID, "null pointer");
    if (!body_ok(body)) return fail(TLMPM_E_INVALID, "body needs mass > 0, moments > 0 and a nonzero quaternion");
    double q[4], nq = 0.0;
    for (int i = 0; i < 4; i++) nq += body->q[i] * body->q[i];
    nq = std::sqrt(nq);
    for (int i = 0; i < 4; i++) q[i] = body->q[i] / nq;
    double R[9];
    quat_rot(q, R);
    tlmpm_tool t;
    memset(&t, 0, sizeof(t));
    t.blade = *bb;
    double r[3];
    mat_vec(R, bb->x_e, r);
    mat_vec(R, bb->n, t.blade.n);
    mat_vec(R, bb->e, t.blade.e);
    mat_vec(R, bb->d, t.blade.d);
    double wr[3];
    cross(body->omega, r, wr);
    for (int a = 0; a < 3; a++) {
        t.blade.x_e[a] = body->x[a] + r[a];
        t.blade.v_e[a] = body->v[a] + wr[a];
        t.x_B[a] = body->x[a];
        t.v_B[a] = body->v[a];
        t.omega_B[a] = body->omega[a];
    }
    t.w_B = 0.0;
    t.flags = flags;
    t.inv_mass = 1.0 / body->mass;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0.0;
            for (int k = 0; k < 3; k++) s += R[3 * i + k] * R[3 * j + k] / body->inertia[k];
            t.inv_inertia[3 * i + j] = s;
        }
    *out = t;
    return TLMPM_OK;
}

// ------------------------------------------------------------------- batches
// Many scenes advanced together: one launch per kernel covers the work items of
// every scene, listed as (scene, block) pairs.  Per-scene parameters stay in
// device memory (SceneK / SceneD arrays); the tools of a call, their counts and the
// wrench accumulators of all scenes sit in the batch's own arrays, so a call costs
// one upload and (with a wrench) one download.
namespace {
struct BatchTools {
    DevTool t[TL_MAX_TOOLS];
    int tinfo[4];
};

struct BatchPlan {
    size_t Ks, Ds, tools, wacc, items[TL_ITEM_KINDS], total;
    int n_items[TL_ITEM_KINDS];
};

int ceil_div(long long a, int b) { return (int)((a + b - 1) / b); }

// work items of each kind for one scene of n_active bricks
void items_of(long long n_active, long long n_bricks, long long NN, long long N, int material_contact,
              int pair_blocks, int xcap, int n[TL_ITEM_KINDS])
{
    n[IT_BRICK] = (int)n_active;
    n[IT_NODE] = ceil_div(NN, 256);
    n[IT_CELL] = material_contact ? ceil_div(n_bricks * TL_CELLS, 256) : 0;
    n[IT_WRENCH] = TL_MAX_TOOLS * 6;
    n[IT_SCENE] = 1;
    n[IT_PART] = ceil_div(N, 256);
    n[IT_BFLAG] = ceil_div(n_bricks, 256);
    n[IT_PAIR] = material_contact ? pair_blocks : 0;
    n[IT_XBRICK] = n_active > 0 ? xcap : 0;
}

void scene_items(const tlmpm_scene* sc, int n[TL_ITEM_KINDS])
{
    const SceneK& K = sc->K;
    items_of(sc->D.n_active, (long long)K.cbx * K.cby * K.cbz, K.NN, K.N, K.material_contact, K.pair_blocks, K.xcap,
             n);
}

tlmpm_status batch_plan(tlmpm_scene* const* scenes, int n, BatchPlan& P)
{
    Layout L;
    P.Ks = L.take((size_t)n * sizeof(SceneK));
    P.Ds = L.take((size_t)n * sizeof(SceneD));
    P.tools = L.take((size_t)n * sizeof(BatchTools));
    P.wacc = L.take((size_t)n * TL_MAX_TOOLS * 6 * sizeof(double));
    long long tot[TL_ITEM_KINDS] = {0};
    for (int s = 0; s < n; s++) {
        int c[TL_ITEM_KINDS];
        scene_items(scenes[s], c);
        for (int k = 0; k < TL_ITEM_KINDS; k++) tot[k] += c[k];
    }
    for (int k = 0; k < TL_ITEM_KINDS; k++) {
        if (tot[k] >= (1LL << 31)) return fail(TLMPM_E_INVALID, "batch too large");
        P.n_items[k] = (int)tot[k];
        P.items[k] = L.take((size_t)tot[k] * sizeof(int2));
    }
    P.total = L.take(0) + 256;
    return TLMPM_OK;
}

tlmpm_status check_members(tlmpm_scene* const* scenes, int n)
{
    if (n <= 0 || !scenes) return fail(TLMPM_E_INVALID, "a batch needs at least one scene");
    for (int s = 0; s < n; s++) {
        if (!scenes[s]) return fail(TLMPM_E_INVALID, "null scene in batch");
        if (scenes[s]->K.stencil == 1)
            return fail(TLMPM_E_INVALID, "scenes with the quadratic stencil run one per call (not in a batch)");
        if (scenes[s]->in_batch) return fail(TLMPM_E_INVALID, "scene already belongs to a live batch");
        for (int t = 0; t < s; t++)
            if (scenes[t] == scenes[s]) return fail(TLMPM_E_INVALID, "scene listed twice in batch");
    }
    return TLMPM_OK;
}
} // namespace

// Host staging of the batches built on a device's static scratch: static arrays,
// so that such a batch allocates no pinned memory; one batch per device at a time.
namespace {
struct StaticStaging {
    BatchTools tools[TL_STATIC_MAX_SCENES];
    double wacc[TL_STATIC_MAX_SCENES * TL_MAX_TOOLS * 6];
};
StaticStaging g_static_staging[TL_STATIC_DEVICES];
bool g_static_held[TL_STATIC_DEVICES];
std::mutex g_static_mutex;
} // namespace

struct tlmpm_batch {
    std::vector<tlmpm_scene*> sc;
    int static_dev = -1; // device whose static scratch and staging this batch holds, else -1
    hipStream_t st;
    TlLaunch L;
    BatchTools* d_tools;
    double* d_wacc;
    BatchTools* h_tools = nullptr; // pinned staging of the per-call tools
    double* h_wacc = nullptr;
    hipEvent_t up_done = nullptr;  // the last upload from h_tools finished
    Timing prof;
    GraphCache graphs;
    Fork fork;
    ~tlmpm_batch()
    {
        if (static_dev >= 0) {
            std::lock_guard<std::mutex> lk(g_static_mutex);
            g_static_held[static_dev] = false;
            return;
        }
        if (h_tools) (void)hipHostFree(h_tools);
        if (h_wacc) (void)hipHostFree(h_wacc);
        if (up_done) (void)hipEventDestroy(up_done);
    }
    int cur, rsb;
    bool pending;
};

extern "C" tlmpm_status tlmpm_batch_footprint(tlmpm_scene* const* scenes, int32_t n_scenes, size_t* device_bytes)
{
    if (tlmpm_status r = check_members(scenes, n_scenes)) return r;
    if (!device_bytes) return fail(TLMPM_E_INVALID, "null output");
    BatchPlan P;
    if (tlmpm_status r = batch_plan(scenes, n_scenes, P)) return r;
    *device_bytes = P.total;
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_batch_scene_bytes(const tlmpm_scene_desc* desc, size_t* device_bytes)
{
    tlmpm_status s = validate(desc);
    if (s) return s;
    if (!device_bytes) return fail(TLMPM_E_INVALID, "null output");
    const Dims g = dims_of(desc);
    const long long na = count_active(desc);
    int c[TL_ITEM_KINDS];
    const tlmpm_tuning tun = tuning_now();
    items_of(na, g.n_bricks, g.NN, g.N, desc->material_contact != 0, pair_blocks_of(g.N, tun), xcap_of(na, tun), c);
    size_t b = sizeof(SceneK) + sizeof(SceneD) + sizeof(BatchTools) + TL_MAX_TOOLS * 6 * sizeof(double);
    for (int k = 0; k < TL_ITEM_KINDS; k++) b += (size_t)c[k] * sizeof(int2);
    // the alignment of the batch layout's 4 + TL_ITEM_KINDS arrays and its tail
    b += (4 + TL_ITEM_KINDS) * 255 + 256;
    *device_bytes = b;
    return TLMPM_OK;
}

// static_dev >= 0: ws is that device's static scratch, already held for this batch
// (released by the batch, or here on failure), staging from the static arrays.
static tlmpm_status batch_create(tlmpm_scene* const* scenes, int32_t n_scenes, void* ws, size_t bytes,
                                 void* hip_stream, tlmpm_batch** out, int static_dev)
{
    auto release = [&]() {
        if (static_dev < 0) return;
        std::lock_guard<std::mutex> lk(g_static_mutex);
        g_static_held[static_dev] = false;
    };
    if (tlmpm_status r = check_members(scenes, n_scenes)) return release(), r;
    if (!out) return release(), fail(TLMPM_E_INVALID, "null output");
    *out = nullptr;
    BatchPlan P;
    if (tlmpm_status r = batch_plan(scenes, n_scenes, P)) return release(), r;
    if (static_dev >= 0 && (P.total > TL_STATIC_SCRATCH_BYTES || n_scenes > TL_STATIC_MAX_SCENES))
        return release(), fail(TLMPM_E_NOMEM, "batch needs " + std::to_string(P.total) + " bytes over " +
                                                  std::to_string(n_scenes) + " scenes; the static scratch holds " +
                                                  std::to_string((size_t)TL_STATIC_SCRATCH_BYTES) + " bytes and " +
                                                  std::to_string(TL_STATIC_MAX_SCENES) + " scenes");
    if (!ws || bytes < P.total) return release(), fail(TLMPM_E_NOMEM, "workspace smaller than tlmpm_batch_footprint()");

    // common slot-table state: that of the scenes with a pending F update (the
    // first one's); scenes in another state apply their F update alone, and scenes
    // without a pending update take their tables to the common buffer
    int cur = scenes[0]->cur, rsb = scenes[0]->cur;
    bool pending = false;
    for (int s = 0; s < n_scenes; s++)
        if (scenes[s]->f_pending) {
            cur = scenes[s]->cur;
            rsb = scenes[s]->rsb;
            pending = true;
            break;
        }
    for (int s = 0; s < n_scenes; s++) {
        tlmpm_scene* sc = scenes[s];
        if (sc->f_pending && (sc->cur != cur || sc->rsb != rsb))
            if (tlmpm_status r = flush_F(sc)) return release(), r;
        if (!sc->f_pending && sc->cur != cur) {
            const TlLaunch L1 = single_launch(sc);
            hipError_t e = tl_launch_slots(&L1, cur, sc->cur, 0);
            if (e != hipSuccess) return release(), fail(TLMPM_E_DEVICE, std::string("slot tables: ") + hipGetErrorString(e));
            sc->cur = cur;
        }
        if (!sc->f_pending) sc->rsb = rsb;
    }
    for (int s = 0; s < n_scenes; s++) {
        hipError_t e = hipStreamSynchronize(scenes[s]->st);
        if (e != hipSuccess) return release(), fail(TLMPM_E_DEVICE, std::string("scene stream: ") + hipGetErrorString(e));
    }

    tlmpm_batch* b = new tlmpm_batch();
    b->static_dev = static_dev; // from here the batch releases the hold
    b->sc.assign(scenes, scenes + n_scenes);
    b->st = (hipStream_t)hip_stream;
    b->prof.st = b->st;
    b->cur = cur;
    b->rsb = rsb;
    b->pending = pending;
    char* base = (char*)ws;
    b->d_tools = (BatchTools*)(base + P.tools);
    b->d_wacc = (double*)(base + P.wacc);
    TlLaunch& L = b->L;
    memset(&L, 0, sizeof(L));
    L.Ks = (const SceneK*)(base + P.Ks);
    L.Ds = (const SceneD*)(base + P.Ds);
    L.st = b->st;
    std::vector<SceneK> hk(n_scenes);
    std::vector<SceneD> hd(n_scenes);
    std::vector<int2> items[TL_ITEM_KINDS];
    for (int s = 0; s < n_scenes; s++) {
        const tlmpm_scene* sc = scenes[s];
        hk[s] = sc->K;
        hd[s] = sc->D;
        hd[s].tools = b->d_tools[s].t;
        hd[s].tinfo = b->d_tools[s].tinfo;
        hd[s].wacc = b->d_wacc + (size_t)s * TL_MAX_TOOLS * 6;
        L.any_material |= sc->K.material_contact;
        L.general |= general_path(sc->K);
        int c[TL_ITEM_KINDS];
        scene_items(sc, c);
        for (int k = 0; k < TL_ITEM_KINDS; k++)
            for (int i = 0; i < c[k]; i++) items[k].push_back(make_int2(s, i));
    }
    auto bail = [&](hipError_t e, const char* what) {
        delete b;
        return fail(TLMPM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    hipError_t e;
    if ((e = hipMemcpyAsync(base + P.Ks, hk.data(), n_scenes * sizeof(SceneK), hipMemcpyHostToDevice, b->st)) !=
        hipSuccess)
        return bail(e, "upload scene parameters");
    if ((e = hipMemcpyAsync(base + P.Ds, hd.data(), n_scenes * sizeof(SceneD), hipMemcpyHostToDevice, b->st)) !=
        hipSuccess)
        return bail(e, "upload scene pointers");
    for (int k = 0; k < TL_ITEM_KINDS; k++) {
        L.items[k] = (const int2*)(base + P.items[k]);
        L.n_items[k] = P.n_items[k];
        if (!items[k].empty() &&
            (e = hipMemcpyAsync(base + P.items[k], items[k].data(), items[k].size() * sizeof(int2),
                                hipMemcpyHostToDevice, b->st)) != hipSuccess)
            return bail(e, "upload work items");
    }
    if (static_dev >= 0) {
        // pageable staging: batch_step waits for the batch's stream before reusing it
        b->h_tools = g_static_staging[static_dev].tools;
        b->h_wacc = g_static_staging[static_dev].wacc;
    } else {
        if ((e = hipHostMalloc((void**)&b->h_tools, n_scenes * sizeof(BatchTools), hipHostMallocDefault)) !=
            hipSuccess)
            return bail(e, "pinned staging");
        if ((e = hipHostMalloc((void**)&b->h_wacc, n_scenes * TL_MAX_TOOLS * 6 * sizeof(double),
                               hipHostMallocDefault)) != hipSuccess)
            return bail(e, "pinned staging");
        if ((e = hipEventCreateWithFlags(&b->up_done, hipEventDisableTiming)) != hipSuccess) return bail(e, "event");
    }

    if ((e = hipStreamSynchronize(b->st)) != hipSuccess) return bail(e, "create batch");
    for (tlmpm_scene* sc : b->sc) sc->in_batch = 1;
    *out = b;
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_batch_create(tlmpm_scene* const* scenes, int32_t n_scenes, void* ws, size_t bytes,
                                           void* hip_stream, tlmpm_batch** out)
{
    return batch_create(scenes, n_scenes, ws, bytes, hip_stream, out, -1);
}

extern "C" tlmpm_status tlmpm_batch_create_static(tlmpm_scene* const* scenes, int32_t n_scenes, void* hip_stream,
                                                  tlmpm_batch** out)
{
    if (out) *out = nullptr;
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= TL_STATIC_DEVICES)
        return fail(TLMPM_E_INVALID, "static scratch exists for devices 0.." + std::to_string(TL_STATIC_DEVICES - 1));
    void* ptr = nullptr;
    HIPCHK(tl_static_scratch(dev, &ptr)); // first call on this device: hipGetSymbolAddress
    {
        std::lock_guard<std::mutex> lk(g_static_mutex);
        if (g_static_held[dev])
            return fail(TLMPM_E_INVALID, "the static scratch of device " + std::to_string(dev) +
                                             " is held by a live batch (destroy it first)");
        g_static_held[dev] = true;
    }
    return batch_create(scenes, n_scenes, ptr, TL_STATIC_SCRATCH_BYTES, hip_stream, out, dev);
}

extern "C" tlmpm_status tlmpm_batch_destroy(tlmpm_batch* b)
{
    if (!b) return fail(TLMPM_E_INVALID, "null batch");
    hipError_t e = hipStreamSynchronize(b->st);
    for (tlmpm_scene* sc : b->sc) sc->in_batch = 0;
    delete b;
    if (e != hipSuccess) return fail(TLMPM_E_DEVICE, std::string("destroy batch: ") + hipGetErrorString(e));
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_batch_step(tlmpm_batch* b, const tlmpm_tool* tools, const int32_t* n_tools,
                                         int32_t n_substeps, double* wrench)
{
    if (!b || !n_tools || n_substeps < 0) return fail(TLMPM_E_INVALID, "bad arguments");
    const int n = (int)b->sc.size();
    for (int s = 0; s < n; s++)
        if (n_tools[s] < 0 || n_tools[s] > TL_MAX_TOOLS || (n_tools[s] > 0 && !tools))
            return fail(TLMPM_E_INVALID, "bad tool count (at most 4 tools per scene)");
    // staging free again: the last upload from it finished (pageable staging of a
    // batch on static scratch: the whole stream)
    if (b->up_done)
        HIPCHK(hipEventSynchronize(b->up_done));
    else
        HIPCHK(hipStreamSynchronize(b->st));
    CallFlags f;
    for (int s = 0; s < n; s++) {
        tlmpm_status r = convert_tools(b->sc[s], n_tools[s] ? tools + (size_t)s * TL_MAX_TOOLS : nullptr, n_tools[s],
                                       b->h_tools[s].t, b->h_tools[s].tinfo, f);
        if (r) return fail(r, "scene " + std::to_string(s) + ": " + g_err);
    }
    HIPCHK(hipMemcpyAsync(b->d_tools, b->h_tools, n * sizeof(BatchTools), hipMemcpyHostToDevice, b->st));
    if (b->up_done) HIPCHK(hipEventRecord(b->up_done, b->st));
    HIPCHK(b->fork.init());
    Exec X;
    X.L = b->L;
    X.prof = &b->prof;
    X.fork = &b->fork;
    X.cur = b->cur;
    X.rsb = b->rsb;
    X.pending = b->pending;
    tlmpm_status r = run_substeps(X, n_substeps, f, &b->graphs);
    b->cur = X.cur;
    b->rsb = X.rsb;
    b->pending = X.pending;
    for (tlmpm_scene* sc : b->sc) {
        sc->cur = X.cur;
        sc->rsb = X.rsb;
        if (n_substeps > 0) sc->f_pending = true;
    }
    if (r) return r;
    if (wrench) {
        const size_t per = TL_MAX_TOOLS * 6;
        if (f.any_contact_tool) {
            HIPCHK(hipMemcpyAsync(b->h_wacc, b->d_wacc, n * per * sizeof(double), hipMemcpyDeviceToHost, b->st));
            HIPCHK(hipStreamSynchronize(b->st));
        }
        const double inv = n_substeps > 0 ? 1.0 / n_substeps : 0.0;
        for (int s = 0; s < n; s++)
            for (size_t q = 0; q < per; q++)
                wrench[s * per + q] =
                    (f.any_contact_tool && (int)q < n_tools[s] * 6) ? b->h_wacc[s * per + q] * inv : 0.0;
    }
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_batch_sync(tlmpm_batch* b)
{
    if (!b) return fail(TLMPM_E_INVALID, "null batch");
    HIPCHK(hipStreamSynchronize(b->st));
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_batch_profile_enable(tlmpm_batch* b, int32_t enable)
{
    if (!b) return fail(TLMPM_E_INVALID, "null batch");
    b->prof.on = enable == 1;
    b->prof.xfer = enable == 2;
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_batch_profile_read(tlmpm_batch* b, int32_t n_classes, double* ms, int64_t* launches)
{
    if (!b) return fail(TLMPM_E_INVALID, "null batch");
    return timing_read(b->prof, n_classes, ms, launches);
}

extern "C" tlmpm_status tlmpm_batch_set_graphs(tlmpm_batch* b, int32_t enable)
{
    if (!b) return fail(TLMPM_E_INVALID, "null batch");
    b->graphs.on = enable != 0;
    return TLMPM_OK;
}

// ------------------------------------------------------------ surface (Sec. III-F)
namespace {
SurfGrid surf_grid(const tlmpm_scene* sc)
{
    SurfGrid G;
    G.sx = 2 * sc->K.cx;
    G.sy = 2 * sc->K.cy;
    G.sz = 2 * sc->K.cz;
    G.S = (long long)G.sx * G.sy * G.sz;
    G.C = (long long)(G.sx + 1) * (G.sy + 1) * (G.sz + 1);
    G.ox = sc->K.ox;
    G.oy = sc->K.oy;
    G.oz = sc->K.oz;
    G.h = 0.5 * sc->K.dx;
    return G;
}

struct SurfLayout {
    size_t head, smap, creg, voff, qoff, bsum, vX, vp, vw, vcode, vx, quads, qcut, total;
};

// the tables of the lattice first (their size depends on the grid only), then the
// vertex and quad arrays
SurfLayout surf_layout(const SurfGrid& G, long long nv, long long nq)
{
    Layout L;
    SurfLayout o;
    o.head = L.take(2 * sizeof(long long));
    o.smap = L.take((size_t)G.S * 8);
    o.creg = L.take((size_t)G.C * 4);
    o.voff = L.take((size_t)(G.C + 1) * 4);
    o.qoff = L.take((size_t)(G.S + 1) * 4);
    const long long nb = (std::max(G.C, G.S) + 1023) / 1024;
    o.bsum = L.take((size_t)(nb + 1) * 4);
    o.vX = L.take((size_t)nv * 16);
    o.vp = L.take((size_t)nv * 32);
    o.vw = L.take((size_t)nv * 32);
    o.vcode = L.take((size_t)nv * 4);
    o.vx = L.take((size_t)nv * 16);
    o.quads = L.take((size_t)nq * 16);
    o.qcut = L.take((size_t)nq);
    o.total = L.take(0) + 256;
    return o;
}

SurfMem surf_mem(void* ws, const SurfLayout& o)
{
    char* b = (char*)ws;
    SurfMem M;
    M.smap = (unsigned long long*)(b + o.smap);
    M.creg = (uint32_t*)(b + o.creg);
    M.voff = (int*)(b + o.voff);
    M.qoff = (int*)(b + o.qoff);
    M.bsum = (int*)(b + o.bsum);
    M.vX = (float4*)(b + o.vX);
    M.vp = (int*)(b + o.vp);
    M.vw = (float*)(b + o.vw);
    M.vcode = (uint32_t*)(b + o.vcode);
    M.vx = (float4*)(b + o.vx);
    M.quads = (int4*)(b + o.quads);
    M.qcut = (uint8_t*)(b + o.qcut);
    return M;
}
} // namespace

extern "C" tlmpm_status tlmpm_surface_footprint(tlmpm_scene* sc, size_t* bytes)
{
    if (!sc || !bytes) return fail(TLMPM_E_INVALID, "bad arguments");
    *bytes = surf_layout(surf_grid(sc), 0, 0).total;
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_surface_build(tlmpm_scene* sc, void* ws, size_t bytes, int64_t counts[2],
                                            size_t* needed)
{
    if (!sc || !counts || !needed) return fail(TLMPM_E_INVALID, "bad arguments");
    if (tlmpm_status r = refuse_batched(sc)) return r;
    const SurfGrid G = surf_grid(sc);
    const SurfLayout base = surf_layout(G, 0, 0);
    if (G.S >= (1LL << 31) || G.C >= (1LL << 31)) return fail(TLMPM_E_INVALID, "site lattice too large");
    if (!ws || bytes < base.total) return fail(TLMPM_E_NOMEM, "workspace smaller than tlmpm_surface_footprint()");
    const SurfMem M0 = surf_mem(ws, base);
    HIPCHK(tl_surface_count(&sc->K, &sc->D, &G, &M0, sc->st));
    int nvq[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(&nvq[0], M0.voff + G.C, 4, hipMemcpyDeviceToHost, sc->st));
    HIPCHK(hipMemcpyAsync(&nvq[1], M0.qoff + G.S, 4, hipMemcpyDeviceToHost, sc->st));
    HIPCHK(hipStreamSynchronize(sc->st));
    counts[0] = nvq[0];
    counts[1] = nvq[1];
    const SurfLayout full = surf_layout(G, nvq[0], nvq[1]);
    *needed = full.total;
    if (bytes < full.total)
        return fail(TLMPM_E_NOMEM, "the surface needs " + std::to_string(full.total) + " bytes of workspace");
    const SurfMem M = surf_mem(ws, full);
    HIPCHK(tl_surface_fill(&sc->K, &sc->D, &G, &M, sc->st));
    const long long head[2] = {nvq[0], nvq[1]};
    HIPCHK(hipMemcpyAsync((char*)ws + full.head, head, sizeof(head), hipMemcpyHostToDevice, sc->st));
    HIPCHK(hipStreamSynchronize(sc->st));
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_surface_read(tlmpm_scene* sc, const void* ws, size_t bytes, float* x, float* X,
                                           uint64_t* code, int32_t* quads, uint8_t* cut)
{
    if (!sc || !ws) return fail(TLMPM_E_INVALID, "bad arguments");
    if (tlmpm_status r = refuse_batched(sc)) return r;
    const SurfGrid G = surf_grid(sc);
    long long head[2] = {0, 0};
    if (bytes < surf_layout(G, 0, 0).total) return fail(TLMPM_E_NOMEM, "workspace smaller than the surface's");
    HIPCHK(hipMemcpyAsync(head, ws, sizeof(head), hipMemcpyDeviceToHost, sc->st));
    HIPCHK(hipStreamSynchronize(sc->st));
    const long long nv = head[0], nq = head[1];
    const SurfLayout o = surf_layout(G, nv, nq);
    if (nv < 0 || nq < 0 || bytes < o.total) return fail(TLMPM_E_INVALID, "workspace does not hold a built surface");
    const SurfMem M = surf_mem(const_cast<void*>(ws), o);
    if (x) HIPCHK(tl_surface_embed(&sc->K, &sc->D, &M, (int)nv, sc->st));
    std::vector<float4> f4;
    if (x || X) f4.resize((size_t)nv);
    auto copy4 = [&](const float4* src, float* dst) -> tlmpm_status {
        if (nv) HIPCHK(hipMemcpyAsync(f4.data(), src, (size_t)nv * 16, hipMemcpyDeviceToHost, sc->st));
        HIPCHK(hipStreamSynchronize(sc->st));
        for (long long i = 0; i < nv; i++) {
            dst[3 * i] = f4[i].x;
            dst[3 * i + 1] = f4[i].y;
            dst[3 * i + 2] = f4[i].z;
        }
        return TLMPM_OK;
    };
    if (x)
        if (tlmpm_status r = copy4(M.vx, x)) return r;
    if (X)
        if (tlmpm_status r = copy4(M.vX, X)) return r;
    if (code) {
        std::vector<uint32_t> c((size_t)nv);
        if (nv) HIPCHK(hipMemcpyAsync(c.data(), M.vcode, (size_t)nv * 4, hipMemcpyDeviceToHost, sc->st));
        HIPCHK(hipStreamSynchronize(sc->st));
        for (long long i = 0; i < nv; i++) code[i] = code_to_ternary(c[i], sc->max_cuts);
    }
    if (quads) {
        if (nq) HIPCHK(hipMemcpyAsync(quads, M.quads, (size_t)nq * 16, hipMemcpyDeviceToHost, sc->st));
        HIPCHK(hipStreamSynchronize(sc->st));
    }
    if (cut) {
        if (nq) HIPCHK(hipMemcpyAsync(cut, M.qcut, (size_t)nq, hipMemcpyDeviceToHost, sc->st));
        HIPCHK(hipStreamSynchronize(sc->st));
    }
    return TLMPM_OK;
}
