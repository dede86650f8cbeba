// tlmpm_contact.hip -- material-material contact (Sec. III-E, Eqs. 10-13).
//
// Candidates: a particle whose 3x3x3 block of reference cells holds an empty or
// out-of-grid cell, or a particle whose side code conflicts with its own.  The
// conflict test uses one OR-ed code per cell: p conflicts with some particle of a
// cell iff (s1_p & OR s2) | (s2_p & OR s1) != 0.
//
// Pairs are found in the current configuration: candidates are hashed into bins
// of edge h >= every contact reach (R_p + R_q + dt |v_p - v_q|); each hash bucket
// is a list built with 64-bit compare-and-swap on (generation, head), so the table
// is never cleared.  A pair is evaluated by both particles with the same operands
// (the lower sorted index first), so the two impulses are exact negatives; each
// particle sorts its contacts by partner index before summing, which makes the
// result independent of the list order.  The tangential spring of a pair is kept
// by its lower index in a per-particle list (double buffered, stamped by substep).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "tlmpm_common.h"

#define DEV __device__ __forceinline__
#define TL_MAXC 48

DEV uint32_t ckey(const SceneK& S, uint32_t code) { return S.single_field ? 0u : (code & TL_CODE_MASK); }

DEV bool cconflict(uint32_t a, uint32_t b)
{
    uint32_t a1 = a & 0x7FFFu, a2 = (a >> 15) & 0x7FFFu;
    uint32_t b1 = b & 0x7FFFu, b2 = (b >> 15) & 0x7FFFu;
    return ((a1 & b2) | (a2 & b1)) != 0u;
}

// cell slot (sorted order) of global cell (x, y, z); -1 outside the grid
DEV long long cell_slot(const SceneK& S, int x, int y, int z)
{
    if (x < 0 || y < 0 || z < 0 || x >= S.cx || y >= S.cy || z >= S.cz) return -1;
    long long brick = ((long long)(z >> 2) * S.cby + (y >> 2)) * S.cbx + (x >> 2);
    int lx = x & 3, ly = y & 3, lz = z & 3;
    int w = (lx & 1) | ((ly & 1) << 1) | ((lz & 1) << 2);
    int i = (lx >> 1) | ((ly >> 1) << 1) | ((lz >> 1) << 2);
    return brick * TL_CELLS + w * 8 + i;
}

DEV void slot_cell(const SceneK& S, long long cs, int& x, int& y, int& z)
{
    long long brick = cs / TL_CELLS;
    int r = (int)(cs % TL_CELLS), w = r >> 3, i = r & 7;
    int bx = (int)(brick % S.cbx), by = (int)((brick / S.cbx) % S.cby), bz = (int)(brick / ((long long)S.cbx * S.cby));
    x = bx * TL_B + 2 * (i & 1) + (w & 1);
    y = by * TL_B + 2 * ((i >> 1) & 1) + ((w >> 1) & 1);
    z = bz * TL_B + 2 * ((i >> 2) & 1) + ((w >> 2) & 1);
}

// per cell: OR of the particles' codes; at creation also the static surface flag
__global__ void k_cellmask(SceneK S, SceneD D, long long n_slots, int with_static)
{
    long long cs = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cs >= n_slots) return;
    uint32_t m = 0;
    for (int p = D.cell_start[cs]; p < D.cell_start[cs + 1]; p++) m |= ckey(S, D.code[p]);
    D.cmask[cs] = m;
    if (with_static) {
        int x, y, z;
        slot_cell(S, cs, x, y, z);
        uint8_t st = 0;
        if (x < S.cx && y < S.cy && z < S.cz)
            for (int dz = -1; dz <= 1; dz++)
                for (int dy = -1; dy <= 1; dy++)
                    for (int dx = -1; dx <= 1; dx++) {
                        long long o = cell_slot(S, x + dx, y + dy, z + dz);
                        if (o < 0 || D.cell_start[o + 1] == D.cell_start[o]) st = 1;
                    }
        D.cstatic[cs] = st;
    }
}

// candidate bit of every particle; per brick: whether it holds a candidate
__global__ __launch_bounds__(256) void k_cand(SceneK S, SceneD D)
{
    const int brick = D.active[blockIdx.x];
    const int bx = brick % S.cbx, by = (brick / S.cbx) % S.cby, bz = brick / (S.cbx * S.cby);
    bool any = false;
    for (int c = threadIdx.x / 8; c < TL_CELLS; c += blockDim.x / 8) {
        long long cs = (long long)brick * TL_CELLS + c;
        int w = c >> 3, i = c & 7;
        int x = bx * TL_B + 2 * (i & 1) + (w & 1);
        int y = by * TL_B + 2 * ((i >> 1) & 1) + ((w >> 1) & 1);
        int z = bz * TL_B + 2 * ((i >> 2) & 1) + ((w >> 2) & 1);
        uint32_t nm = 0; // OR of the codes around the cell
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    long long o = cell_slot(S, x + dx, y + dy, z + dz);
                    if (o >= 0) nm |= D.cmask[o];
                }
        const bool st = D.cstatic[cs] != 0;
        for (int p = D.cell_start[cs] + (threadIdx.x & 7); p < D.cell_start[cs + 1]; p += 8) {
            uint32_t code = D.code[p];
            bool cand = st || cconflict(ckey(S, code), nm);
            uint32_t nc = cand ? (code | TL_CAND_BIT) : (code & ~TL_CAND_BIT);
            if (nc != code) D.code[p] = nc;
            any |= cand;
        }
    }
    int a = __syncthreads_or(any);
    if (threadIdx.x == 0) D.bcand[brick] = a;
}

// bin edge from the largest speed of any brick (conservative reach)
__global__ void k_hsize(SceneK S, SceneD D)
{
    __shared__ float s[256];
    float m = 0.0f;
    for (int b = threadIdx.x; b < D.n_active; b += blockDim.x) m = fmaxf(m, D.aabb[(long long)D.active[b] * 8 + 6]);
    s[threadIdx.x] = m;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] = fmaxf(s[threadIdx.x], s[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        float h = (2.0f * S.Rmax + 2.0f * S.dt * s[0]) * 1.001f + 1e-7f;
        D.hbin[0] = fmaxf(h, 0.25f * (float)S.dx);
    }
}

DEV void bin_of(const float x[3], float inv_h, int b[3])
{
    for (int a = 0; a < 3; a++) b[a] = (int)floorf(x[a] * inv_h);
}

DEV uint32_t bin_hash(int i, int j, int k, uint32_t mask)
{
    return (((uint32_t)i * 73856093u) ^ ((uint32_t)j * 19349663u) ^ ((uint32_t)k * 83492791u)) & mask;
}

DEV void cur_pos(const SceneK& S, const SceneD& D, long long p, float x[3])
{
    x[0] = D.X[p] + D.u[p];
    x[1] = D.X[S.N + p] + D.u[S.N + p];
    x[2] = D.X[2 * S.N + p] + D.u[2 * S.N + p];
}

__global__ __launch_bounds__(256) void k_bin_insert(SceneK S, SceneD D, unsigned gen)
{
    const int brick = D.active[blockIdx.x];
    if (!D.bcand[brick]) return;
    const float inv_h = 1.0f / D.hbin[0];
    const int beg = D.cell_start[(long long)brick * TL_CELLS], end = D.cell_start[(long long)(brick + 1) * TL_CELLS];
    for (int p = beg + threadIdx.x; p < end; p += blockDim.x) {
        if (!(D.code[p] & TL_CAND_BIT)) continue;
        float x[3];
        cur_pos(S, D, p, x);
        int b[3];
        bin_of(x, inv_h, b);
        uint32_t h = bin_hash(b[0], b[1], b[2], D.hmask);
        unsigned long long* slot = (unsigned long long*)&D.htab[h];
        unsigned long long old = *slot, nv;
        do {
            unsigned og = (unsigned)(old >> 32);
            int head = (og == gen) ? (int)(old & 0xFFFFFFFFull) : -1;
            D.hnext[p] = head;
            __threadfence();
            nv = ((unsigned long long)gen << 32) | (unsigned)p;
            unsigned long long prev = atomicCAS(slot, old, nv);
            if (prev == old) break;
            old = prev;
        } while (true);
    }
}

DEV void friction_f(const SceneK& S, const float vrel[3], const float n[3], float fn, float meff, float u[3],
                    float ft[3])
{
    float dt = S.dt;
    float un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2];
    float up[3] = {u[0] - un * n[0], u[1] - un * n[1], u[2] - un * n[2]};
    float lu = sqrtf(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    float lp = sqrtf(up[0] * up[0] + up[1] * up[1] + up[2] * up[2]);
    float sc = lp > 0.0f ? lu / lp : 0.0f;
    float ut[3] = {up[0] * sc, up[1] * sc, up[2] * sc};
    float vn = vrel[0] * n[0] + vrel[1] * n[1] + vrel[2] * n[2];
    float vt[3] = {vrel[0] - vn * n[0], vrel[1] - vn * n[1], vrel[2] - vn * n[2]};
    float kt = S.gamma_k * meff / (dt * dt);
    float ct = 2.0f * S.gamma_c * sqrtf(meff * kt);
    float ftr[3] = {-kt * ut[0] - ct * vt[0], -kt * ut[1] - ct * vt[1], -kt * ut[2] - ct * vt[2]};
    float lf = sqrtf(ftr[0] * ftr[0] + ftr[1] * ftr[1] + ftr[2] * ftr[2]);
    if (lf <= S.mu_s * fn) {
        for (int a = 0; a < 3; a++) {
            ft[a] = ftr[a];
            u[a] = ut[a] + dt * vt[a];
        }
    } else {
        float sl = S.mu_d * fn / lf;
        for (int a = 0; a < 3; a++) {
            ft[a] = ftr[a] * sl;
            u[a] = -(ft[a] + ct * vt[a]) / kt;
        }
    }
}

struct PState {
    float x[3], v[3], m, R;
};

DEV PState load_pstate(const SceneK& S, const SceneD& D, long long p)
{
    PState s;
    cur_pos(S, D, p, s.x);
    s.v[0] = D.v[p];
    s.v[1] = D.v[S.N + p];
    s.v[2] = D.v[2 * S.N + p];
    s.m = S.m_uniform ? S.m0 : D.m[p];
    float V0 = S.v_uniform ? S.V0 : D.V0[p];
    s.R = 0.5f * S.s_R * cbrtf(V0);
    return s;
}

// Pair impulse on the owner o (lower index) from r, Eqs. 10-12; u is the owner's
// spring (in: old, out: new).  Returns false when the pair is not in contact.
DEV bool pair_impulse(const SceneK& S, const PState& o, const PState& r, float u[3], float J[3])
{
    const float dt = S.dt;
    float dx[3] = {o.x[0] - r.x[0], o.x[1] - r.x[1], o.x[2] - r.x[2]};
    float dist = sqrtf(dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]);
    if (!(dist > 0.0f)) return false;
    float n[3] = {dx[0] / dist, dx[1] / dist, dx[2] / dist};
    float vrel[3] = {o.v[0] - r.v[0], o.v[1] - r.v[1], o.v[2] - r.v[2]};
    float vn = vrel[0] * n[0] + vrel[1] * n[1] + vrel[2] * n[2];
    float dhat = o.R + r.R - (dist + fminf(dt * vn, 0.0f));
    float meff = o.m * r.m / (o.m + r.m);
    float fn = S.s_n * meff / (dt * dt) * fmaxf(dhat, 0.0f);
    if (!(fn > 0.0f)) return false;
    float ft[3];
    friction_f(S, vrel, n, fn, meff, u, ft);
    for (int a = 0; a < 3; a++) J[a] = (fn * n[a] + ft[a]) * dt;
    return true;
}

DEV void ref_cell(const SceneK& S, const SceneD& D, long long p, int c[3])
{
    c[0] = (int)floor(((double)D.X[p] - S.ox) / S.dx);
    c[1] = (int)floor(((double)D.X[S.N + p] - S.oy) / S.dx);
    c[2] = (int)floor(((double)D.X[2 * S.N + p] - S.oz) / S.dx);
}

__global__ __launch_bounds__(128) void k_pairs(SceneK S, SceneD D, unsigned gen, int hold, int hnew, int stamp)
{
    const int brick = D.active[blockIdx.x];
    if (!D.bcand[brick]) return;
    const float inv_h = 1.0f / D.hbin[0];
    const long long N = S.N;
    const int beg = D.cell_start[(long long)brick * TL_CELLS], end = D.cell_start[(long long)(brick + 1) * TL_CELLS];
    for (int p = beg + threadIdx.x; p < end; p += blockDim.x) {
        uint32_t code = D.code[p];
        if (!(code & TL_CAND_BIT)) continue;
        const uint32_t kp = ckey(S, code);
        PState sp = load_pstate(S, D, p);
        int cp[3];
        ref_cell(S, D, p, cp);
        int b[3];
        bin_of(sp.x, inv_h, b);
        int nq = 0;
        int qs[TL_MAXC];
        float Js[TL_MAXC][3];
        float Us[TL_MAXC][3];
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    int bb[3] = {b[0] + dx, b[1] + dy, b[2] + dz};
                    uint32_t h = bin_hash(bb[0], bb[1], bb[2], D.hmask);
                    unsigned long long e = D.htab[h];
                    if ((unsigned)(e >> 32) != gen) continue;
                    for (int q = (int)(e & 0xFFFFFFFFull); q >= 0; q = D.hnext[q]) {
                        if (q == p) continue;
                        PState sq = load_pstate(S, D, q);
                        int bq[3];
                        bin_of(sq.x, inv_h, bq);
                        if (bq[0] != bb[0] || bq[1] != bb[1] || bq[2] != bb[2]) continue; // hash collision
                        uint32_t kq = ckey(S, D.code[q]);
                        int cq[3];
                        ref_cell(S, D, q, cq);
                        bool near = abs(cp[0] - cq[0]) <= 1 && abs(cp[1] - cq[1]) <= 1 && abs(cp[2] - cq[2]) <= 1;
                        if (near && !cconflict(kp, kq)) continue; // reading R17 exclusion
                        const bool own = p < q;
                        const int o = own ? p : q, r = own ? q : p;
                        // owner's old spring for this partner
                        float u[3] = {0.0f, 0.0f, 0.0f};
                        int hdr = D.ph_n[(long long)hold * N + o];
                        if ((hdr >> 8) == stamp - 1) {
                            int cnt = hdr & 0xFF;
                            const int* ql = D.ph_q + ((long long)hold * N + o) * TL_PCAP;
                            for (int k = 0; k < cnt; k++)
                                if (ql[k] == r) {
                                    const float* ul = D.ph_u + (((long long)hold * N + o) * TL_PCAP + k) * 3;
                                    u[0] = ul[0];
                                    u[1] = ul[1];
                                    u[2] = ul[2];
                                    break;
                                }
                        }
                        float J[3];
                        bool hit = own ? pair_impulse(S, sp, sq, u, J) : pair_impulse(S, sq, sp, u, J);
                        if (!hit) continue;
                        if (nq == TL_MAXC) {
                            atomicOr(D.status, TL_ST_CONTACT);
                            continue;
                        }
                        qs[nq] = q;
                        for (int a = 0; a < 3; a++) {
                            Js[nq][a] = own ? J[a] : -J[a];
                            Us[nq][a] = u[a];
                        }
                        nq++;
                    }
                }
        // order by partner index, then sum (independent of the bucket list order)
        for (int a = 1; a < nq; a++) {
            int key = qs[a];
            float j0 = Js[a][0], j1 = Js[a][1], j2 = Js[a][2], u0 = Us[a][0], u1 = Us[a][1], u2 = Us[a][2];
            int c = a - 1;
            while (c >= 0 && qs[c] > key) {
                qs[c + 1] = qs[c];
                Js[c + 1][0] = Js[c][0];
                Js[c + 1][1] = Js[c][1];
                Js[c + 1][2] = Js[c][2];
                Us[c + 1][0] = Us[c][0];
                Us[c + 1][1] = Us[c][1];
                Us[c + 1][2] = Us[c][2];
                c--;
            }
            qs[c + 1] = key;
            Js[c + 1][0] = j0;
            Js[c + 1][1] = j1;
            Js[c + 1][2] = j2;
            Us[c + 1][0] = u0;
            Us[c + 1][1] = u1;
            Us[c + 1][2] = u2;
        }
        float Jt[3] = {0.0f, 0.0f, 0.0f};
        int nown = 0;
        int* ql = D.ph_q + ((long long)hnew * N + p) * TL_PCAP;
        float* ul = D.ph_u + ((long long)hnew * N + p) * TL_PCAP * 3;
        for (int k = 0; k < nq; k++) {
            Jt[0] += Js[k][0];
            Jt[1] += Js[k][1];
            Jt[2] += Js[k][2];
            if (p < qs[k]) {
                if (nown < TL_PCAP) {
                    ql[nown] = qs[k];
                    ul[nown * 3 + 0] = Us[k][0];
                    ul[nown * 3 + 1] = Us[k][1];
                    ul[nown * 3 + 2] = Us[k][2];
                    nown++;
                } else {
                    atomicOr(D.status, TL_ST_CONTACT);
                }
            }
        }
        D.ph_n[(long long)hnew * N + p] = (stamp << 8) | nown;
        D.Jmat[p] = Jt[0];
        D.Jmat[N + p] = Jt[1];
        D.Jmat[2 * N + p] = Jt[2];
    }
}

extern "C" {
hipError_t tl_launch_cellmask(const SceneK* S, const SceneD* D, long long n_slots, int with_static, hipStream_t st)
{
    if (n_slots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cellmask, dim3((unsigned)((n_slots + 255) / 256)), dim3(256), 0, st, *S, *D, n_slots,
                       with_static);
    return hipGetLastError();
}

hipError_t tl_launch_cand(const SceneK* S, const SceneD* D, hipStream_t st)
{
    if (D->n_active == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cand, dim3(D->n_active), dim3(256), 0, st, *S, *D);
    return hipGetLastError();
}

hipError_t tl_launch_contact(const SceneK* S, const SceneD* D, unsigned gen, int hold, int hnew, int stamp,
                             hipStream_t st)
{
    if (D->n_active == 0) return hipSuccess;
    hipLaunchKernelGGL(k_hsize, dim3(1), dim3(256), 0, st, *S, *D);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_insert, dim3(D->n_active), dim3(256), 0, st, *S, *D, gen);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pairs, dim3(D->n_active), dim3(128), 0, st, *S, *D, gen, hold, hnew, stamp);
    return hipGetLastError();
}
}
