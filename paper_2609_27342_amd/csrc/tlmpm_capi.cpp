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
#include <string>
#include <vector>

#include "../../include/tlmpm.h"
#include "tlmpm_common.h"

extern "C" {
hipError_t tl_launch_p2g(const SceneK*, const SceneD*, int, int, int, int, int, int, hipStream_t);
hipError_t tl_launch_rigid(const SceneK*, const SceneD*, int, int, double, int, hipStream_t);
hipError_t tl_launch_mixed(const SceneK*, const SceneD*, int, hipStream_t);
hipError_t tl_launch_g2p(const SceneK*, const SceneD*, int, hipStream_t);
hipError_t tl_launch_labels(const SceneK*, const SceneD*, int, double, int, hipStream_t);
hipError_t tl_launch_slots(const SceneK*, const SceneD*, int, int, int, hipStream_t);
hipError_t tl_launch_fill_f32(float*, long long, float, hipStream_t);
hipError_t tl_launch_fill_i32(int*, long long, int, hipStream_t);
hipError_t tl_launch_aabb(const SceneK*, const SceneD*, hipStream_t);
hipError_t tl_launch_wrench(const SceneD*, int, hipStream_t);
hipError_t tl_launch_cellmask(const SceneK*, const SceneD*, long long, int, int, hipStream_t);
hipError_t tl_launch_cand(const SceneK*, const SceneD*, int, hipStream_t);
hipError_t tl_launch_contact(const SceneK*, const SceneD*, unsigned, int, int, int, hipStream_t);
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

struct tlmpm_scene {
    SceneK K;
    SceneD D;
    hipStream_t st;
    int max_cuts;
    int n_bricks;
    int cur;       // slot table in use
    int rsb;       // slot table of the pending re-scatter
    bool f_pending;
    int stamp;
    int hist_buf = 0;   // pair-spring buffer written last
    std::vector<int> active_host;
    // kernel timing (diagnostics)
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, int>> ev_used; // (class, first event index)
    size_t ev_next = 0;
};

// Brackets one launch with events when profiling is on.
struct ProfScope {
    tlmpm_scene* sc;
    int cls;
    int idx = -1;
    ProfScope(tlmpm_scene* s, int c) : sc(s), cls(c)
    {
        if (!sc->prof) return;
        while (sc->ev_pool.size() < sc->ev_next + 2) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            sc->ev_pool.push_back(e);
        }
        idx = (int)sc->ev_next;
        sc->ev_next += 2;
        (void)hipEventRecord(sc->ev_pool[idx], sc->st);
    }
    ~ProfScope()
    {
        if (idx < 0) return;
        (void)hipEventRecord(sc->ev_pool[idx + 1], sc->st);
        sc->ev_used.push_back({cls, idx});
    }
};

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
    size_t X, u, v, H, code, code_prev, D, perm, E, m, V0, cell_start, active, cnt0, cnt1, sc0, sc1, p2g, rs, hist,
        aabb, wpart, wacc, Jmat, Jrig, brig, bmixed, tools, status, dirty, bdirty, pcell, cand_idx, cmask, cstatic, bcand, hbin, bcount, bids, cslot, brec, htab, hnext, orec, ph_n, ph_q, ph_u,
        total;
    uint32_t hmask;
};

Offsets plan(const tlmpm_scene_desc* d)
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
    o.sc0 = L.take((size_t)g.NN * TL_SCAP * 4);
    o.sc1 = L.take((size_t)g.NN * TL_SCAP * 4);
    o.p2g = L.take((size_t)g.NN * 8 * TL_SCAP * 8 * f); // 7 components padded to 8
    o.rs = L.take((size_t)g.NN * 8 * TL_SCAP * 4 * f);
    o.hist = L.take((size_t)(TL_MAX_TOOLS + 1) * 4 * N * f);
    o.aabb = L.take((size_t)g.n_bricks * 8 * f);
    o.wpart = L.take((size_t)g.n_bricks * TL_MAX_TOOLS * 6 * f);
    o.wacc = L.take(TL_MAX_TOOLS * 6 * sizeof(double));
    o.Jmat = d->material_contact ? L.take(3 * N * f) : 0;
    o.Jrig = L.take(3 * N * f);
    o.brig = L.take((size_t)g.n_bricks * 4);
    o.bmixed = L.take((size_t)g.n_bricks * 4);
    o.tools = L.take(TL_MAX_TOOLS * sizeof(DevTool));
    o.hmask = 0;
    if (d->material_contact) {
        size_t cells = (size_t)g.n_bricks * TL_CELLS;
        o.cmask = L.take(cells * 4);
        o.cstatic = L.take(cells);
        o.bcand = L.take((size_t)g.n_bricks * 4);
        o.cand_idx = L.take(N * 4);
        o.hbin = L.take(4);
        size_t buckets = 4096;
        while (buckets < N / 2) buckets <<= 1;
        o.hmask = (uint32_t)(buckets - 1);
        o.bcount = L.take(buckets * 4);
        o.bids = L.take(buckets * TL_BCAP * 4);
        o.cslot = L.take(N * 4);
        o.brec = L.take(buckets * TL_BCAP * 48);
        o.htab = L.take(buckets * 8);
        o.hnext = L.take(N * 4);
        o.orec = L.take(N * 48);
        o.ph_n = L.take(2 * N * 4);
        o.ph_q = L.take(2 * N * TL_PCAP * 4);
        o.ph_u = L.take(2 * N * TL_PCAP * 3 * f);
    }
    o.status = L.take(4);
    o.dirty = L.take(4);
    o.bdirty = L.take((size_t)g.n_bricks * 4);
    o.pcell = L.take(N * 4);
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
    *device_bytes = plan(desc).total;
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_create_scene(const tlmpm_scene_desc* d, void* ws, size_t bytes, void* hip_stream,
                                           tlmpm_scene** out)
{
    tlmpm_status s = validate(d);
    if (s) return s;
    if (!out) return fail(TLMPM_E_INVALID, "null output");
    *out = nullptr;
    Offsets o = plan(d);
    if (!ws || bytes < o.total) return fail(TLMPM_E_NOMEM, "workspace smaller than tlmpm_scene_footprint()");
    Dims g = dims_of(d);
    const long long N = g.N;

    // reference cell of every particle (FP64, the same formula as the bricks use)
    std::vector<long long> key(N);
    std::vector<int> cnt((size_t)g.n_bricks * TL_CELLS + 1, 0);
    for (long long p = 0; p < N; p++) {
        int c[3];
        for (int a = 0; a < 3; a++) {
            double q = ((double)d->X[3 * p + a] - d->origin[a]) / d->dx;
            double fl = std::floor(q);
            if (!(fl >= 0.0) || fl >= (double)d->cells[a])
                return fail(TLMPM_E_INVALID, "particle " + std::to_string(p) + " lies outside the reference grid");
            c[a] = (int)fl;
        }
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
    std::vector<int> active;
    for (long long b = 0; b < g.n_bricks; b++)
        if (cell_start[(b + 1) * TL_CELLS] > cell_start[b * TL_CELLS]) active.push_back((int)b);

    tlmpm_scene* sc = new tlmpm_scene();
    sc->st = (hipStream_t)hip_stream;
    sc->max_cuts = d->max_cuts;
    sc->n_bricks = (int)g.n_bricks;
    sc->cur = 0;
    sc->rsb = 0;
    sc->f_pending = false;
    sc->stamp = 1;
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
    D.hist = (float*)(base + o.hist);
    D.aabb = (float*)(base + o.aabb);
    D.wpart = (float*)(base + o.wpart);
    D.wacc = (double*)(base + o.wacc);
    D.Jmat = d->material_contact ? (float*)(base + o.Jmat) : nullptr;
    D.Jrig = (float*)(base + o.Jrig);
    D.brig = (int*)(base + o.brig);
    D.bmixed = (int*)(base + o.bmixed);
    D.tools = (DevTool*)(base + o.tools);
    if (d->material_contact) {
        D.cmask = (uint32_t*)(base + o.cmask);
        D.cstatic = (uint8_t*)(base + o.cstatic);
        D.bcand = (int*)(base + o.bcand);
        D.cand_idx = (int*)(base + o.cand_idx);
        D.hbin = (float*)(base + o.hbin);
        D.hmask = o.hmask;
        D.bcount = (int*)(base + o.bcount);
        D.bids = (int*)(base + o.bids);
        D.cslot = (int*)(base + o.cslot);
        D.brec = (float4*)(base + o.brec);
        D.htab = (unsigned long long*)(base + o.htab);
        D.hnext = (int*)(base + o.hnext);
        D.orec = (float4*)(base + o.orec);
        D.ph_n = (int*)(base + o.ph_n);
        D.ph_q = (int*)(base + o.ph_q);
        D.ph_u = (float*)(base + o.ph_u);
    }
    D.status = (int*)(base + o.status);
    D.dirty = (int*)(base + o.dirty);
    D.bdirty = (int*)(base + o.bdirty);
    D.pcell = (int*)(base + o.pcell);

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
    // rigid-contact history stamps start invalid
    if ((e = tl_launch_fill_f32(D.hist, (long long)(TL_MAX_TOOLS + 1) * 4 * N, 0.0f, sc->st)) != hipSuccess)
        return bail(e, "init history");
    if ((e = tl_launch_slots(&K, &D, 0, 0, 1, sc->st)) != hipSuccess) return bail(e, "slot table");
    if ((e = tl_launch_aabb(&K, &D, sc->st)) != hipSuccess) return bail(e, "aabb");
    if (d->material_contact) {
        if ((e = tl_launch_cellmask(&K, &D, g.n_bricks * TL_CELLS, 1, 1, sc->st)) != hipSuccess)
            return bail(e, "cell masks");
        if ((e = tl_launch_cand(&K, &D, 1, sc->st)) != hipSuccess) return bail(e, "candidates");
    }
    if ((e = hipStreamSynchronize(sc->st)) != hipSuccess) return bail(e, "create");
    *out = sc;
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_profile_enable(tlmpm_scene* sc, int32_t enable)
{
    if (!sc) return fail(TLMPM_E_INVALID, "null scene");
    sc->prof = enable != 0;
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_profile_read(tlmpm_scene* sc, int32_t n_classes, double* ms, int64_t* launches)
{
    if (!sc || n_classes < 0 || n_classes > 6 || (n_classes && (!ms || !launches)))
        return fail(TLMPM_E_INVALID, "bad arguments");
    HIPCHK(hipStreamSynchronize(sc->st));
    for (int c = 0; c < n_classes; c++) {
        ms[c] = 0.0;
        launches[c] = 0;
    }
    for (auto& u : sc->ev_used) {
        float t = 0.0f;
        HIPCHK(hipEventElapsedTime(&t, sc->ev_pool[u.second], sc->ev_pool[u.second + 1]));
        if (u.first < n_classes) {
            ms[u.first] += t;
            launches[u.first] += 1;
        }
    }
    sc->ev_used.clear();
    sc->ev_next = 0;
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_destroy_scene(tlmpm_scene* sc)
{
    if (!sc) return fail(TLMPM_E_INVALID, "null scene");
    for (hipEvent_t e : sc->ev_pool) (void)hipEventDestroy(e);
    hipError_t e = hipStreamSynchronize(sc->st);
    delete sc;
    if (e != hipSuccess) return fail(TLMPM_E_DEVICE, std::string("destroy: ") + hipGetErrorString(e));
    return TLMPM_OK;
}

// contact candidates after a change of side codes (bricks flagged in bdirty, or
// everything when forced)
static tlmpm_status refresh_candidates(tlmpm_scene* sc, int force)
{
    if (!sc->K.material_contact) return TLMPM_OK;
    ProfScope ps(sc, 4);
    HIPCHK(tl_launch_cellmask(&sc->K, &sc->D, (long long)sc->n_bricks * TL_CELLS, 0, force, sc->st));
    HIPCHK(tl_launch_cand(&sc->K, &sc->D, force, sc->st));
    return TLMPM_OK;
}

// label pass over the tools in D.tools flagged TL_TOOL_LABELS, then slot-table
// maintenance (no host synchronisation)
static tlmpm_status label_pass(tlmpm_scene* sc, int n_tools, double jdt, bool any_new)
{
    SceneD& D = sc->D;
    if (any_new) {
        ProfScope ps(sc, 5);
        HIPCHK(tl_launch_fill_f32(D.D, sc->K.N, 0.0f, sc->st));
    }
    {
        ProfScope ps(sc, 2);
        HIPCHK(tl_launch_labels(&sc->K, &D, n_tools, jdt, sc->f_pending ? 1 : 0, sc->st));
    }
    {
        ProfScope ps(sc, 3);
        HIPCHK(tl_launch_mixed(&sc->K, &D, 0, sc->st));
    }
    int dst = (sc->f_pending && sc->cur == sc->rsb) ? 1 - sc->cur : sc->cur;
    {
        ProfScope ps(sc, 3);
        HIPCHK(tl_launch_slots(&sc->K, &D, dst, sc->cur, 0, sc->st));
    }
    sc->cur = dst;
    tlmpm_status rs = refresh_candidates(sc, 0);
    if (rs) return rs;
    HIPCHK(tl_launch_fill_i32(D.dirty, 1, 0, sc->st));
    HIPCHK(tl_launch_fill_i32(D.bdirty, sc->n_bricks, 0, sc->st));
    return TLMPM_OK;
}

static tlmpm_status upload_tools(tlmpm_scene* sc, const DevTool* t, int n)
{
    if (n > 0) HIPCHK(hipMemcpyAsync(sc->D.tools, t, n * sizeof(DevTool), hipMemcpyHostToDevice, sc->st));
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_assign_labels(tlmpm_scene* sc, const tlmpm_blade* blades, int32_t n_blades)
{
    if (!sc || (n_blades > 0 && !blades) || n_blades < 0 || n_blades > TL_MAX_TOOLS)
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
    tlmpm_status s = upload_tools(sc, t, n_blades);
    if (s) return s;
    return label_pass(sc, n_blades, 0.0, any_new);
}

static tlmpm_status flush_F(tlmpm_scene* sc)
{
    if (!sc->f_pending) return TLMPM_OK;
    HIPCHK(tl_launch_p2g(&sc->K, &sc->D, 1, 0, 0, sc->cur, sc->rsb, 0, sc->st));
    sc->f_pending = false;
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_step(tlmpm_scene* sc, const tlmpm_tool* tools, int32_t n_tools, int32_t n_substeps,
                                   double* wrench)
{
    if (!sc || n_tools < 0 || n_tools > TL_MAX_TOOLS || (n_tools > 0 && !tools) || n_substeps < 0)
        return fail(TLMPM_E_INVALID, "bad arguments (at most 4 tools)");
    for (int t = 0; t < n_tools; t++) {
        const tlmpm_blade& B = tools[t].blade;
        if (!frame_ok(B)) return fail(TLMPM_E_INVALID, "tool frame (n, e, d) must be orthonormal");
        if ((tools[t].flags & TLMPM_TOOL_LABELS) && (B.cut_index < 0 || B.cut_index >= sc->max_cuts))
            return fail(TLMPM_E_INVALID, "cut_index out of range");
        if ((tools[t].flags & TLMPM_TOOL_ADVANCE) &&
            (tools[t].omega_B[0] != 0 || tools[t].omega_B[1] != 0 || tools[t].omega_B[2] != 0))
            return fail(TLMPM_E_INVALID, "TLMPM_TOOL_ADVANCE supports translating tools only");
    }
    SceneD& D = sc->D;
    DevTool dtl[TL_MAX_TOOLS];
    memset(dtl, 0, sizeof(dtl));
    bool any_contact_tool = false, any_labels = false, any_new = false;
    for (int t = 0; t < n_tools; t++) {
        const tlmpm_tool& T = tools[t];
        DevTool& o = dtl[t];
        o.b = dev_blade(T.blade);
        for (int a = 0; a < 3; a++) {
            o.xB[a] = T.x_B[a];
            o.vB[a] = T.v_B[a];
            o.wB[a] = (float)T.omega_B[a];
        }
        o.invm = (float)T.w_B;
        o.flags = T.flags;
        o.slot = 1 + t;
        any_contact_tool |= (T.flags & TLMPM_TOOL_CONTACT) != 0;
        any_labels |= (T.flags & TLMPM_TOOL_LABELS) != 0;
        any_new |= (T.flags & TLMPM_TOOL_LABELS) && T.blade.new_cut;
    }
    const bool do_contact = any_contact_tool || sc->K.floor_on;
    {
        tlmpm_status s = upload_tools(sc, dtl, n_tools);
        if (s) return s;
    }
    if (any_contact_tool) HIPCHK(hipMemsetAsync(D.wacc, 0, TL_MAX_TOOLS * 6 * sizeof(double), sc->st));
    for (int j = 0; j < n_substeps; j++) {
        const double jdt = (double)j * sc->K.dt_d;
        if (any_labels) {
            tlmpm_status s = label_pass(sc, n_tools, jdt, any_new && j == 0);
            if (s) return s;
        }
        if (sc->K.material_contact) {
            ProfScope ps(sc, 4);
            int hnew = 1 - sc->hist_buf;
            HIPCHK(tl_launch_contact(&sc->K, &D, (unsigned)sc->stamp, sc->hist_buf, hnew, sc->stamp, sc->st));
            sc->hist_buf = hnew;
        }
        if (do_contact) {
            ProfScope ps(sc, 5);
            HIPCHK(tl_launch_rigid(&sc->K, &D, n_tools, any_contact_tool ? 1 : 0, jdt, sc->stamp, sc->st));
        }
        if (any_contact_tool) {
            ProfScope ps(sc, 5);
            HIPCHK(tl_launch_wrench(&D, n_tools, sc->st));
        }
        const bool differ = sc->f_pending && sc->cur != sc->rsb;
        {
            ProfScope ps(sc, 0);
            HIPCHK(tl_launch_p2g(&sc->K, &D, sc->f_pending ? 1 : 0, 1, differ ? 1 : 0, sc->cur, sc->rsb,
                                 do_contact ? 1 : 0, sc->st));
        }
        {
            ProfScope ps(sc, 1);
            HIPCHK(tl_launch_g2p(&sc->K, &D, sc->cur, sc->st));
        }
        sc->f_pending = true;
        sc->rsb = sc->cur;
        sc->stamp++;
    }
    if (wrench && n_tools > 0) {
        double acc[TL_MAX_TOOLS * 6];
        if (any_contact_tool) {
            HIPCHK(hipMemcpyAsync(acc, D.wacc, n_tools * 6 * sizeof(double), hipMemcpyDeviceToHost, sc->st));
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
    if (!sc || !status) return fail(TLMPM_E_INVALID, "bad arguments");
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
    if (!sc || (mask && !out)) return fail(TLMPM_E_INVALID, "bad arguments");
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
    for (uint32_t bit = 1; bit <= TLMPM_FIELD_DIGITS; bit <<= 1) {
        if (!(mask & bit)) continue;
        void* dst = out[slot++];
        if (!dst) return fail(TLMPM_E_INVALID, "null output buffer");
        if (bit == TLMPM_FIELD_X || bit == TLMPM_FIELD_U || bit == TLMPM_FIELD_V || bit == TLMPM_FIELD_F ||
            bit == TLMPM_FIELD_D) {
            int comps = bit == TLMPM_FIELD_F ? 9 : (bit == TLMPM_FIELD_D ? 1 : 3);
            const float* src = bit == TLMPM_FIELD_X ? D.X
                               : bit == TLMPM_FIELD_U ? D.u
                               : bit == TLMPM_FIELD_V ? D.v
                               : bit == TLMPM_FIELD_F ? D.H
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
    if (!sc || (mask && !in)) return fail(TLMPM_E_INVALID, "bad arguments");
    if (mask & (TLMPM_FIELD_X | TLMPM_FIELD_CODE)) return fail(TLMPM_E_INVALID, "X and CODE are not writable");
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
    for (uint32_t bit = 1; bit <= TLMPM_FIELD_DIGITS; bit <<= 1) {
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
        int comps = bit == TLMPM_FIELD_F ? 9 : (bit == TLMPM_FIELD_D ? 1 : 3);
        float* dstp = bit == TLMPM_FIELD_U ? D.u : bit == TLMPM_FIELD_V ? D.v : bit == TLMPM_FIELD_F ? D.H : D.D;
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
    if (codes_changed) {
        HIPCHK(tl_launch_mixed(&sc->K, &D, 1, sc->st));
        HIPCHK(tl_launch_slots(&sc->K, &D, sc->cur, sc->cur, 1, sc->st));
        sc->rsb = sc->cur;
        tlmpm_status rs = refresh_candidates(sc, 1);
        if (rs) return rs;
    }
    HIPCHK(tl_launch_aabb(&sc->K, &D, sc->st));
    HIPCHK(hipStreamSynchronize(sc->st));
    return TLMPM_OK;
}

extern "C" tlmpm_status tlmpm_slot_stats(tlmpm_scene* sc, int64_t* total_slots, int32_t* max_per_node)
{
    if (!sc) return fail(TLMPM_E_INVALID, "null scene");
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
