// tlmpm_contact.hip -- material-material contact (Sec. III-E, Eqs. 10-13).
//
// Candidates: a particle whose 3x3x3 block of reference cells holds an empty or
// out-of-grid cell, or a particle whose side code conflicts with its own.  The
// conflict test uses one OR-ed code per cell: p conflicts with some particle of a
// cell iff (s1_p & OR s2) | (s2_p & OR s1) != 0.
//
// Pairs are found in the current configuration: candidates are hashed into bins
// of edge h >= every contact reach (R_p + R_q + dt |v_p - v_q|).  Each candidate's
// record (position, velocity, mass, radius, code, reference cell) is written once
// into a dense array indexed by its global candidate number, which follows the
// particle order; a hash bucket holds up to TL_BCAP of these numbers (in arrival
// order, sorted by the pair pass when it reads them), and an overflow list built
// with 64-bit compare-and-swap on (generation, head), so the table is never
// cleared.  A pair is evaluated by both particles with the same operands
// (the lower sorted index first), so the two impulses are exact negatives; each
// particle sums its contacts in a fixed order (bins, then ranks in the bin), which
// makes the result independent of arrival order.  The tangential spring of a pair
// is kept in both particles' lists (double buffered, stamped by substep).
#include <hip/hip_runtime.h>
#include <math.h>
#include <limits.h>
#include <stdint.h>

#include "tlmpm_common.h"
#include "tlmpm_device.h"
#include "tlmpm_reach.h"

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

// per cell: OR of the particles' codes; at creation also the static surface flag.
// Without `force`, only the cells of bricks whose codes changed are recomputed.
DEV void cellmask_body(const SceneK& S, const SceneD& D, int bi, int with_static, int force)
{
    if (!S.material_contact) return;
    const long long n_slots = (long long)S.cbx * S.cby * S.cbz * TL_CELLS;
    long long cs = (long long)bi * blockDim.x + threadIdx.x;
    if (cs >= n_slots) return;
    if (!force && D.bdirty[cs / TL_CELLS] != D.ctr[0]) return;
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

// Candidate bit of every particle and the brick's candidate list (in particle
// order, stored over the brick's particle range).  Without `force`, only bricks
// next to a brick whose codes changed are recomputed.
// First global candidate index of every active brick (exclusive scan of the
// candidate counts in active-brick order) by one block of TL_SCAN_T threads, in
// chunks of TL_SCAN_T * TL_SCAN_PER counts: each chunk is loaded coalesced into LDS,
// every thread scans TL_SCAN_PER consecutive counts there, the thread totals are
// scanned across the block, and the offsets are stored coalesced.
#define TL_SCAN_T 1024
#define TL_SCAN_PER 8
DEV void scan_offsets(const SceneD& D)
{
    constexpr int T = TL_SCAN_T, CH = T * TL_SCAN_PER;
    __shared__ int s_c[CH];
    __shared__ int s_w[T / 64];
    const int n = D.n_active;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    int carry = 0;
    for (int base = 0; base < n; base += CH) {
#pragma unroll
        for (int k = 0; k < TL_SCAN_PER; k++) {
            const int i = base + k * T + t;
            s_c[k * T + t] = i < n ? D.bcand[i] : 0;
        }
        __syncthreads();
        int loc = 0;
#pragma unroll
        for (int k = 0; k < TL_SCAN_PER; k++) loc += s_c[t * TL_SCAN_PER + k];
        int incl = loc;
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o, 64);
            if (lane >= o) incl += v;
        }
        if (lane == 63) s_w[wv] = incl;
        __syncthreads();
        int before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < T / 64; w++) {
            before += w < wv ? s_w[w] : 0;
            total += s_w[w];
        }
        int run = carry + before + incl - loc;
#pragma unroll
        for (int k = 0; k < TL_SCAN_PER; k++) {
            const int c = s_c[t * TL_SCAN_PER + k];
            s_c[t * TL_SCAN_PER + k] = run;
            run += c;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < TL_SCAN_PER; k++) {
            const int i = base + k * T + t;
            if (i < n) D.coff[i] = s_c[k * T + t];
        }
        carry += total;
        __syncthreads();
    }
    if (t == 0) D.coff[n] = carry;
}

// Exact displacement anchor of a brick from its particles' current u (the midpoint
// and half range of each axis): for a brick that gains its first candidates, which
// the last G2P did not keep an anchor for.  Whole block.
DEV void anchor_exact(const SceneK& S, const SceneD& D, int bi, int brick, int beg, int end)
{
    __shared__ float s_r[4][6];
    const long long N = S.N;
    float r[6] = {1e30f, 1e30f, 1e30f, -1e30f, -1e30f, -1e30f};
    for (int p = beg + threadIdx.x; p < end; p += blockDim.x)
        for (int a = 0; a < 3; a++) {
            const float ua = D.u[a * N + p];
            r[a] = fminf(r[a], ua);
            r[3 + a] = fmaxf(r[3 + a], ua);
        }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int q = 0; q < 6; q++) {
        for (int o = 32; o >= 1; o >>= 1) {
            const float t = __shfl_xor(r[q], o, 64);
            r[q] = q < 3 ? fminf(r[q], t) : fmaxf(r[q], t);
        }
        if (lane == 0) s_r[wv][q] = r[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); w++)
            for (int q = 0; q < 6; q++) r[q] = q < 3 ? fminf(r[q], s_r[w][q]) : fmaxf(r[q], s_r[w][q]);
        float a[3], sp = 0.0f;
        for (int k = 0; k < 3; k++) {
            a[k] = 0.5f * (r[k] + r[3 + k]);
            sp = fmaxf(sp, fmaxf(r[3 + k] - a[k], a[k] - r[k]));
        }
        put_anchor(D, bi, brick, 0, a, sp * (1.0f + 1e-6f));
    }
}

// candidate bits and the ordered candidate list of one brick
DEV void cand_brick(const SceneK& S, const SceneD& D, int bi, int brick, int bx, int by, int bz, uint32_t* s_nm,
                    int* s_st, int* s_wave)
{
    const int had = D.bcand[bi]; // (read before thread 0 rewrites it below)
    if (threadIdx.x < TL_CELLS) {
        const int c = threadIdx.x;
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
        s_nm[c] = nm;
        s_st[c] = D.cstatic[cs];
    }
    __syncthreads();
    const int beg = D.cell_start[(long long)brick * TL_CELLS], end = D.cell_start[(long long)(brick + 1) * TL_CELLS];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int base = 0;
    for (int p0 = beg; p0 < end; p0 += blockDim.x) {
        const int p = p0 + threadIdx.x;
        bool cand = false;
        if (p < end) {
            int c = (int)(D.pcell[p] - (long long)brick * TL_CELLS);
            uint32_t code = D.code[p];
            cand = s_st[c] || cconflict(ckey(S, code), s_nm[c]);
            uint32_t nc = cand ? (code | TL_CAND_BIT) : (code & ~TL_CAND_BIT);
            if (nc != code) D.code[p] = nc;
        }
        // ordered compaction: rank = candidates before p in this chunk
        unsigned long long bal = __ballot(cand);
        int in_wave = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) s_wave[wv] = __popcll(bal);
        __syncthreads();
        int before = base;
        for (int k = 0; k < wv; k++) before += s_wave[k];
        if (cand) D.cand_idx[beg + before + in_wave] = p;
        int tot = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); k++) tot += s_wave[k];
        base += tot;
        __syncthreads();
    }
    // a brick with its first candidates has no displacement anchor from the last G2P
    if (S.pair_skip && base > 0 && had == 0) anchor_exact(S, D, bi, brick, beg, end);
    if (threadIdx.x == 0) D.bcand[bi] = base;
}

DEV void cand_body(const SceneK& S, const SceneD& D, int bi, int force)
{
    if (!S.material_contact) return;
    __shared__ uint32_t s_nm[TL_CELLS];
    __shared__ int s_st[TL_CELLS];
    __shared__ int s_wave[4];
    const int stamp = D.ctr[0];
    const int brick = D.active[bi];
    const int bx = brick % S.cbx, by = (brick / S.cbx) % S.cby, bz = brick / (S.cbx * S.cby);
    // recompute when a brick of the 3x3x3 neighbourhood changed codes in this pass
    int near_change = 0;
    if (threadIdx.x < 27) {
        const int d = threadIdx.x;
        const int x = bx + d % 3 - 1, y = by + (d / 3) % 3 - 1, z = bz + d / 9 - 1;
        if (x >= 0 && y >= 0 && z >= 0 && x < S.cbx && y < S.cby && z < S.cbz)
            near_change = D.bdirty[((long long)z * S.cby + y) * S.cbx + x] == stamp;
    }
    const bool go = __syncthreads_or(near_change) || force;
    if (go) cand_brick(S, D, bi, brick, bx, by, bz, s_nm, s_st, s_wave);
}

// Candidate pass of one scene with TL_CBRICKS bricks per workgroup (bricks w, w + G,
// w + 2G, ... of G workgroups): 27 threads per brick look for a code change in its
// 3x3x3 neighbourhood at once, then the workgroup recomputes the bricks that need it
// one after another.  Far fewer workgroups than bricks, most of which only look.
#define TL_CBRICKS 8
__global__ __launch_bounds__(256) void k_cand_multi(SceneK S, SceneD D, int force)
{
    static_assert(27 * TL_CBRICKS <= 256, "27 threads per brick");
    if (!S.material_contact) return;
    __shared__ uint32_t s_nm[TL_CELLS];
    __shared__ int s_st[TL_CELLS];
    __shared__ int s_wave[4];
    __shared__ int s_go[TL_CBRICKS];
    const int stamp = D.ctr[0];
    const int G = gridDim.x;
    if (threadIdx.x < TL_CBRICKS) s_go[threadIdx.x] = force;
    __syncthreads();
    if (!force && threadIdx.x < 27 * TL_CBRICKS) {
        const int k = threadIdx.x / 27, d = threadIdx.x % 27;
        const int bi = blockIdx.x + k * G;
        if (bi < D.n_active) {
            const int brick = D.active[bi];
            const int bx = brick % S.cbx, by = (brick / S.cbx) % S.cby, bz = brick / (S.cbx * S.cby);
            const int x = bx + d % 3 - 1, y = by + (d / 3) % 3 - 1, z = bz + d / 9 - 1;
            if (x >= 0 && y >= 0 && z >= 0 && x < S.cbx && y < S.cby && z < S.cbz &&
                D.bdirty[((long long)z * S.cby + y) * S.cbx + x] == stamp)
                s_go[k] = 1; // (every writer stores 1)
        }
    }
    __syncthreads();
    for (int k = 0; k < TL_CBRICKS; k++) {
        const int bi = blockIdx.x + k * G;
        if (!s_go[k] || bi >= D.n_active) continue;
        const int brick = D.active[bi];
        const int bx = brick % S.cbx, by = (brick / S.cbx) % S.cby, bz = brick / (S.cbx * S.cby);
        cand_brick(S, D, bi, brick, bx, by, bz, s_nm, s_st, s_wave);
        __syncthreads(); // the brick's LDS words are reused by the next one
    }
}

// one block of TL_SCAN_T threads per scene
DEV void cscan_body(const SceneK& S, const SceneD& D, int bi)
{
    if (S.material_contact) scan_offsets(D);
}


// bin edge from the largest speed (conservative reach of every pair); the speed
// bounds of the bricks were gathered into TL_HSLOTS slots by the G2P pass
DEV float bin_edge(const SceneK& S, const SceneD& D)
{
    static_assert(TL_HSLOTS == 64, "one slot per lane of a wave");
    float vmax = __int_as_float(D.hmax[(threadIdx.x & 63) * TL_HSTRIDE]);
    for (int o = 32; o >= 1; o >>= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, o, 64));
    const float h = (2.0f * S.Rmax + 2.0f * S.dt * vmax) * 1.001f + 1e-7f;
    return fmaxf(h, 0.25f * (float)S.dx);
}

DEV void bin_of(const float x[3], float inv_h, int b[3])
{
    for (int a = 0; a < 3; a++) b[a] = (int)floorf(x[a] * inv_h);
}

DEV uint32_t bin_hash(int i, int j, int k, uint32_t mask)
{
    // 4x4x4 blocks of bins share 64 consecutive buckets, so the 27 bins around a
    // particle touch few cache lines; the block coordinates are hashed
    const uint32_t hb = ((uint32_t)(i >> 2) * 73856093u) ^ ((uint32_t)(j >> 2) * 19349663u) ^
                        ((uint32_t)(k >> 2) * 83492791u);
    return ((hb << 6) | (uint32_t)((i & 3) | ((j & 3) << 2) | ((k & 3) << 4))) & mask;
}

DEV void cur_pos(const SceneK& S, const SceneD& D, long long p, float x[3])
{
    x[0] = D.X[p] + D.u[p];
    x[1] = D.X[S.N + p] + D.u[S.N + p];
    x[2] = D.X[2 * S.N + p] + D.u[2 * S.N + p];
}

// Candidate record: {id, code, reference cell x | y << 16, cell z}, {x, m}, {v, R}
// (three float4; cells per axis are below 2^16).  The first two hold what the pair
// search's filters read (reach, reference-neighbour exclusion, bin), so the third
// is loaded only for the few entries that pass them.
DEV void make_rec(const SceneK& S, const SceneD& D, int p, const float x[3], float4 r[3])
{
    float m = S.m_uniform ? S.m0 : D.m[p];
    float V0 = S.v_uniform ? S.V0 : D.V0[p];
    int c[3];
    slot_cell(S, D.pcell[p], c[0], c[1], c[2]); // reference cell, packed 16 + 16 bits and 16 bits
    r[0] = make_float4(__int_as_float(p), __uint_as_float(D.code[p]), __int_as_float(c[0] | (c[1] << 16)),
                       __int_as_float(c[2]));
    r[1] = make_float4(x[0], x[1], x[2], m);
    r[2] = make_float4(D.v[p], D.v[S.N + p], D.v[2 * S.N + p], 0.5f * S.s_R * cbrtf(V0));
}

// Flag in the fourth word of a candidate record (beside the cell's z, 16 bits): the
// binning found that the candidate has no contact partner this substep, and the pair
// pass writes its zero impulse without searching.
#define TL_REC_SKIP (1 << 30)

// Can a candidate of brick `brick` (active index bi) have a contact partner this
// substep?  Run by the 64 lanes of the first wave; *skip = 1 when no candidate of the
// brick can have one except through a side-key conflict with *orn, the OR of the keys
// of the bricks with candidates among the 27 around it (this one included).  Only
// candidates are partners, so only bricks with candidates enter the bounds; their
// anchors come from the last G2P, or, for a brick that gained its first candidates
// in this substep's candidate pass, from that pass (anchor_exact).  The bounds (pair_skip_bounds_ok):
// the scene's displacement range per axis from the anchors' slot maxima (u in
// [min (a - s), max (a + s)]), and for the 27 bricks |u_p - u_q| <= |a_b - a_b'| +
// s_b + s_b' (|u - a| <= s within a brick).
DEV void pair_skip_test(const SceneK& S, const SceneD& D, int bi, int brick, float hb, int* skip, uint32_t* orn)
{
    const int l = threadIdx.x;
    float um[6];
    for (int f = 0; f < 6; f++) {
        uint32_t k = 0u;
        for (int q = l; q < TL_USLOTS; q += 64) {
            const uint32_t t = D.umm[f * TL_USLOTS + q];
            k = t > k ? t : k;
        }
        for (int o = 32; o >= 1; o >>= 1) {
            const uint32_t t = (uint32_t)__shfl_xor((int)k, o, 64);
            k = t > k ? t : k;
        }
        um[f] = fkey_value(k);
    }
    const int bx = brick % S.cbx, by = (brick / S.cbx) % S.cby, bz = brick / (S.cbx * S.cby);
    float a[3] = {0.0f, 0.0f, 0.0f}, sp = -1.0f;
    uint32_t orr = 0u;
    if (l < 27) {
        const int x = bx + l % 3 - 1, y = by + (l / 3) % 3 - 1, z = bz + l / 9 - 1;
        if (x >= 0 && y >= 0 && z >= 0 && x < S.cbx && y < S.cby && z < S.cbz) {
            const long long nb = ((long long)z * S.cby + y) * S.cbx + x;
            const int nbi = D.bact[nb];
            // only bricks with candidates hold partners (and keep anchors)
            if (nbi >= 0 && D.bcand[nbi] > 0) {
                brick_anchor(S, D, nbi, (int)nb, a, sp);
                orr = D.bor[nb];
            }
        }
    }
    float a0[3];
    for (int k = 0; k < 3; k++) a0[k] = __shfl(a[k], 13, 64);
    const float s0 = __shfl(sp, 13, 64);
    float dk[3];
    for (int k = 0; k < 3; k++) dk[k] = sp >= 0.0f ? fabsf(a[k] - a0[k]) + sp : 0.0f;
    for (int o = 32; o >= 1; o >>= 1) {
        for (int k = 0; k < 3; k++) dk[k] = fmaxf(dk[k], __shfl_xor(dk[k], o, 64));
        orr |= (uint32_t)__shfl_xor((int)orr, o, 64);
    }
    if (l == 0) {
        float bb[7];
        brick_aabb(S, D, bi, brick, bb);
        float M = 0.0f;
        for (int k = 0; k < 6; k++) M = fmaxf(M, fabsf(bb[k]));
        float U[3], Dk[3];
        for (int k = 0; k < 3; k++) {
            U[k] = um[k] + um[3 + k];
            Dk[k] = dk[k] + s0;
        }
        *skip = (s0 >= 0.0f && pair_skip_bounds_ok(U, Dk, hb, (float)S.dx, M)) ? 1 : 0;
        *orn = orr;
    }
}

// Bins the candidates of every brick: each candidate writes its record at its
// global number g; slot = atomicAdd on the bucket count; the first TL_BCAP numbers
// are kept in arrival order, later candidates go to a lock-free overflow list
// (generation-stamped heads, never cleared).  The pair pass sorts a bucket's
// numbers before use, so its result does not depend on the arrival order.
// self_scan: the block sums the candidate counts of the bricks before it itself (no
// scan launch; each block reads up to n_active counts, so only for scenes of few
// bricks), and the last brick's block writes the total for the pair pass.
DEV void bin_insert_body(const SceneK& S, const SceneD& D, int bi, int self_scan = 0)
{
    if (!S.material_contact) return;
    const unsigned gen = (unsigned)D.ctr[0];
    const int brick = D.active[bi];
    const int nc = D.bcand[bi];
    const bool last = self_scan && bi == D.n_active - 1;
    if (!nc && bi != 0 && !last) return;
    const float hb = bin_edge(S, D);
    if (bi == 0 && threadIdx.x == 0) D.hbin[0] = hb; // for the pair pass
    int g0;
    if (self_scan) {
        __shared__ int s_sum[4];
        int a = 0;
        for (int i = threadIdx.x; i < bi; i += blockDim.x) a += D.bcand[i];
        for (int o = 32; o >= 1; o >>= 1) a += __shfl_xor(a, o, 64);
        if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = a;
        __syncthreads();
        g0 = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) g0 += s_sum[w];
        if (threadIdx.x == 0) {
            D.coff[bi] = g0;
            if (last) D.coff[bi + 1] = g0 + nc;
        }
    } else {
        g0 = D.coff[bi];
    }
    if (!nc) return;
    __shared__ int s_skip;
    __shared__ uint32_t s_orn;
    if (S.pair_skip) {
        if (threadIdx.x < 64) pair_skip_test(S, D, bi, brick, hb, &s_skip, &s_orn);
        __syncthreads();
    }
    const bool may_skip = S.pair_skip && s_skip;
    const uint32_t orn = S.pair_skip ? s_orn : 0u;
    const float inv_h = 1.0f / hb;
    const int beg = D.cell_start[(long long)brick * TL_CELLS];
    int* bcount = D.bcount + (gen & 1u) * ((long long)D.hmask + 1); // this substep's counts
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        const int p = D.cand_idx[beg + c];
        const int g = g0 + c;
        float x[3];
        cur_pos(S, D, p, x);
        float4 r[3];
        make_rec(S, D, p, x, r);
        if (may_skip && !cconflict(ckey(S, __float_as_uint(r[0].y)), orn))
            r[0].w = __int_as_float(__float_as_int(r[0].w) | TL_REC_SKIP);
        float4* dst = D.crec + (long long)g * 3;
        dst[0] = r[0];
        dst[1] = r[1];
        dst[2] = r[2];
        int b[3];
        bin_of(x, inv_h, b);
        uint32_t h = bin_hash(b[0], b[1], b[2], D.hmask);
        int slot = atomicAdd(&bcount[h], 1);
        if (slot < TL_BCAP) {
            D.bids[(long long)h * TL_BCAP + slot] = g;
            continue;
        }
        unsigned long long* hs = (unsigned long long*)&D.htab[h];
        unsigned long long old = *hs, nv;
        while (true) {
            unsigned og = (unsigned)(old >> 32);
            D.hnext[g] = (og == gen) ? (int)(old & 0xFFFFFFFFull) : -1;
            nv = ((unsigned long long)gen << 32) | (unsigned)g;
            unsigned long long prev = atomicCAS(hs, old, nv);
            if (prev == old) break;
            old = prev;
        }
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

DEV PState pstate_of(const float4 r[3])
{
    PState s;
    s.x[0] = r[1].x;
    s.x[1] = r[1].y;
    s.x[2] = r[1].z;
    s.m = r[1].w;
    s.v[0] = r[2].x;
    s.v[1] = r[2].y;
    s.v[2] = r[2].z;
    s.R = r[2].w;
    return s;
}

// reference cell of a record (x | y << 16 and z in its first vector)
DEV void rec_cell(const float4& r0, int c[3])
{
    const int xy = __float_as_int(r0.z);
    c[0] = xy & 0xFFFF;
    c[1] = (xy >> 16) & 0xFFFF;
    c[2] = __float_as_int(r0.w) & 0xFFFF;
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

// Pair search and impulses over all candidates of the scene (grid-stride over the
// global candidate list).  TL_PLANES lanes per candidate: lane l fetches the counts
// of neighbour bins l, l + TL_PLANES, ... (of 27); the bins' entries (in particle
// index order) are compacted into one list per candidate in bin order, which the
// lanes visit strided, then the buckets' overflow lists; each lane sums its
// contacts and the lane sums are added by a fixed shuffle tree.  The tangential
// spring of a pair is kept by both particles (each in its own list, oriented for
// the pair's lower index): both sides evaluate the pair with the same operands, so
// the two copies stay equal and no particle reads its partner's list.  A list is
// only searched by partner, so its order does not matter.

// the first c (<= TL_BCAP) candidate numbers of bucket h in increasing order
// (sorting network on eight values; unused places hold INT_MAX)
DEV void bucket_sorted(const SceneD& D, uint32_t h, int c, int e[TL_BCAP])
{
    static_assert(TL_BCAP == 8, "the sorting network below covers 8 entries");
    const int4* row = (const int4*)(D.bids + (long long)h * TL_BCAP);
    const int4 a = row[0];
    const int4 b = c > 4 ? row[1] : make_int4(INT_MAX, INT_MAX, INT_MAX, INT_MAX);
    e[0] = a.x;
    e[1] = c > 1 ? a.y : INT_MAX;
    e[2] = c > 2 ? a.z : INT_MAX;
    e[3] = c > 3 ? a.w : INT_MAX;
    e[4] = b.x;
    e[5] = c > 5 ? b.y : INT_MAX;
    e[6] = c > 6 ? b.z : INT_MAX;
    e[7] = c > 7 ? b.w : INT_MAX;
    auto cx = [&](int i, int j) {
        const int lo = min(e[i], e[j]), hi = max(e[i], e[j]);
        e[i] = lo;
        e[j] = hi;
    };
    cx(0, 1); cx(2, 3); cx(0, 2); cx(1, 3); cx(1, 2); // first four
    if (c > 4) {
        cx(4, 6); cx(5, 7); cx(4, 5); cx(6, 7); cx(5, 6); // last four (sorted 4 + 4, then merged)
        cx(0, 4); cx(1, 5); cx(2, 6); cx(3, 7);
        cx(2, 4); cx(3, 5);
        cx(1, 2); cx(3, 4); cx(5, 6);
    }
}

#define TL_PLIST (TL_PLANES == 8 ? 96 : 64) // compacted neighbour entries per candidate held in LDS
DEV void pairs_body(const SceneK& S, const SceneD& D, int bi)
{
    if (!S.material_contact) return;
    // history stamp of this substep; its parity selects the spring buffer written
    const int stamp = D.ctr[0];
    const unsigned gen = (unsigned)stamp;
    const int hnew = stamp & 1, hold = hnew ^ 1;
    // the binning has read the speed bounds and the displacement bounds: G2P gathers
    // them anew for the next substep
    if (bi == 0) {
        if (threadIdx.x < TL_HSLOTS) D.hmax[threadIdx.x * TL_HSTRIDE] = 0;
        if (S.pair_skip)
            for (int q = threadIdx.x; q < 6 * TL_USLOTS; q += blockDim.x) D.umm[q] = 0u;
    }
    // bucket counts: this substep's buffer, and the other one cleared for the next
    const long long nbk = (long long)D.hmask + 1;
    const int* bcount = D.bcount + (stamp & 1) * nbk;
    {
        int* nxt = D.bcount + ((stamp + 1) & 1) * nbk;
        for (long long i = (long long)bi * blockDim.x + threadIdx.x; i < nbk; i += (long long)S.pair_blocks * blockDim.x)
            nxt[i] = 0;
    }
    __shared__ int s_q[TL_PCAND][TL_PCAP];
    __shared__ float s_u[TL_PCAND][TL_PCAP][3];
    __shared__ int s_nold[TL_PCAND], s_nnew[TL_PCAND];
    __shared__ int s_ids[TL_PCAND][TL_PLIST];          // candidate numbers of the bins' entries
    __shared__ unsigned char s_bin[TL_PCAND][TL_PLIST]; // which of the 27 bins each came from
    const int total = D.coff[D.n_active];
    const float hb = D.hbin[0];
    const float inv_h = 1.0f / hb;
    // no pair farther apart than the bin edge can touch this substep: the edge
    // exceeds R_p + R_q + dt |v_p - v_q| for every pair (see bin_edge)
    const float reach2 = hb * hb;
    const long long N = S.N;
    const int sub = threadIdx.x / TL_PLANES; // candidate of this lane group
    const int l = threadIdx.x % TL_PLANES;   // lane in the group
    constexpr int NBL = (27 + TL_PLANES - 1) / TL_PLANES; // bins per lane
    const int stride = S.pair_blocks * TL_PCAND;
    for (int c0 = bi * TL_PCAND; c0 < total; c0 += stride) {
        const int g = c0 + sub;
        const bool has = g < total;
        float4 rp[3];
        if (has) {
            const float4* src = D.crec + (long long)g * 3;
            rp[0] = src[0];
            rp[1] = src[1];
            rp[2] = src[2];
        }
        const int p = has ? __float_as_int(rp[0].x) : -1;
        // a candidate the binning found without a possible partner: zero impulse, no springs
        const bool look = has && !(__float_as_int(rp[0].w) & TL_REC_SKIP);
        // this lane's bins: l, l + TL_PLANES, ... of the 27 around the candidate
        int bq[3] = {0, 0, 0};
        if (has) {
            const float xp[3] = {rp[1].x, rp[1].y, rp[1].z};
            bin_of(xp, inv_h, bq);
        }
        // distances from the candidate to the faces of its own bin
        float lo[3], hi[3];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const float xa = a == 0 ? rp[1].x : a == 1 ? rp[1].y : rp[1].z;
            lo[a] = xa - (float)bq[a] * hb;
            hi[a] = (float)(bq[a] + 1) * hb - xa;
        }
        uint32_t hq[NBL];
        int cntq[NBL];
#pragma unroll
        for (int j = 0; j < NBL; j++) {
            const int d = l + TL_PLANES * j;
            const int o[3] = {d % 3 - 1, (d / 3) % 3 - 1, d / 9 - 1};
            // a bin whose nearest point is farther than sqrt(0.999) h holds no
            // partner: a contact needs a distance below h / 1.001 (see bin_edge)
            float e2 = 0.0f;
#pragma unroll
            for (int a = 0; a < 3; a++) {
                const float e = o[a] < 0 ? lo[a] : o[a] > 0 ? hi[a] : 0.0f;
                e2 += e * e;
            }
            hq[j] = bin_hash(bq[0] + o[0], bq[1] + o[1], bq[2] + o[2], D.hmask);
            cntq[j] = (look && d < 27 && e2 < 0.999f * reach2) ? bcount[hq[j]] : 0;
        }
        // the candidate's springs of the last substep, staged in LDS
        int nold = 0;
        if (look) {
            const int hdr = D.ph_n[(long long)hold * N + p];
            if ((hdr >> 8) == stamp - 1) nold = min(hdr & 0xFF, TL_PCAP);
        }
        for (int k = l; k < nold; k += TL_PLANES) {
            const long long e = (long long)hold * N * TL_PCAP + (long long)p * TL_PCAP + k;
            s_q[sub][k] = D.ph_q[e];
            s_u[sub][k][0] = D.ph_u[e * 3 + 0];
            s_u[sub][k][1] = D.ph_u[e * 3 + 1];
            s_u[sub][k][2] = D.ph_u[e * 3 + 2];
        }
        if (l == 0) {
            s_nold[sub] = nold;
            s_nnew[sub] = 0;
        }
        // inline entries of the 27 bins in bin order, compacted into one list per
        // candidate (the first TL_PLIST of them; the rest are visited by the lane
        // that owns their bin)
        // list position of the first entry of bin d = l + TL_PLANES j: the entries of the
        // rows j' < j in every lane, plus those of row j in the lanes below l
        int pos[NBL], n_list = 0;
#pragma unroll
        for (int j = 0; j < NBL; j++) {
            const int c = min(cntq[j], TL_BCAP);
            int incl = c;
#pragma unroll
            for (int o = 1; o < TL_PLANES; o <<= 1) {
                const int t = __shfl_up(incl, o, TL_PLANES);
                if (l >= o) incl += t;
            }
            pos[j] = n_list + incl - c;
            n_list += __shfl(incl, TL_PLANES - 1, TL_PLANES);
        }
#pragma unroll
        for (int j = 0; j < NBL; j++) {
            const int c = min(cntq[j], TL_BCAP);
            if (c == 0) continue;
            const int d = l + TL_PLANES * j;
            int e[TL_BCAP];
            bucket_sorted(D, hq[j], c, e);
#pragma unroll
            for (int k = 0; k < TL_BCAP; k++) {
                const int at = pos[j] + k;
                if (k < c && at < TL_PLIST) {
                    s_ids[sub][at] = e[k];
                    s_bin[sub][at] = (unsigned char)d;
                }
            }
        }
        __syncthreads();
        float Jt[3] = {0.0f, 0.0f, 0.0f};
        if (look) {
            const uint32_t kp = ckey(S, __float_as_uint(rp[0].y));
            const PState sp = pstate_of(rp);
            int cp[3];
            rec_cell(rp[0], cp);
            int* ql_new = D.ph_q + ((long long)hnew * N + p) * TL_PCAP;
            float* ul_new = D.ph_u + ((long long)hnew * N + p) * TL_PCAP * 3;
            // entry src of bin d, its first two vectors r0, r1 already loaded
            auto visit = [&](const float4* src, const float4& r0, const float4& r1, int d) {
                const int q = __float_as_int(r0.x);
                if (q == p) return;
                {
                    const float ex = sp.x[0] - r1.x, ey = sp.x[1] - r1.y, ez = sp.x[2] - r1.z;
                    if (ex * ex + ey * ey + ez * ez >= reach2) return;
                }
                uint32_t kq = ckey(S, __float_as_uint(r0.y));
                int cq[3];
                rec_cell(r0, cq);
                bool near = abs(cp[0] - cq[0]) <= 1 && abs(cp[1] - cq[1]) <= 1 && abs(cp[2] - cq[2]) <= 1;
                if (near && !cconflict(kp, kq)) return; // reading R17 exclusion
                {
                    const float xq[3] = {r1.x, r1.y, r1.z};
                    int bz[3];
                    bin_of(xq, inv_h, bz);
                    // hash collision: the entry's own bin is not the probed one
                    if (bz[0] != bq[0] + d % 3 - 1 || bz[1] != bq[1] + (d / 3) % 3 - 1 || bz[2] != bq[2] + d / 9 - 1)
                        return;
                }
                const float4 rec[3] = {r0, r1, src[2]};
                PState sq = pstate_of(rec);
                const bool own = p < q;
                // the pair's spring of the last substep
                float u[3] = {0.0f, 0.0f, 0.0f};
                for (int k = 0; k < s_nold[sub]; k++)
                    if (s_q[sub][k] == q) {
                        u[0] = s_u[sub][k][0];
                        u[1] = s_u[sub][k][1];
                        u[2] = s_u[sub][k][2];
                        break;
                    }
                float J[3];
                bool hit = own ? pair_impulse(S, sp, sq, u, J) : pair_impulse(S, sq, sp, u, J);
                if (!hit) return;
                const float sg = own ? 1.0f : -1.0f;
                Jt[0] += sg * J[0];
                Jt[1] += sg * J[1];
                Jt[2] += sg * J[2];
                int k = atomicAdd(&s_nnew[sub], 1);
                if (k < TL_PCAP) {
                    ql_new[k] = q;
                    ul_new[k * 3 + 0] = u[0];
                    ul_new[k * 3 + 1] = u[1];
                    ul_new[k * 3 + 2] = u[2];
                } else {
                    atomicOr(D.status, TL_ST_CONTACT);
                }
            };
            // the list, strided over the lanes, two independent records at a time
            const int nl = min(n_list, TL_PLIST);
            for (int i = l; i < nl; i += 2 * TL_PLANES) {
                const int i2 = i + TL_PLANES;
                const bool two = i2 < nl;
                const float4* s1 = D.crec + (long long)s_ids[sub][i] * 3;
                const float4* s2 = D.crec + (long long)s_ids[sub][two ? i2 : i] * 3;
                const float4 a0 = s1[0], a1 = s1[1], b0 = s2[0], b1 = s2[1];
                visit(s1, a0, a1, s_bin[sub][i]);
                if (two) visit(s2, b0, b1, s_bin[sub][i2]);
            }
            // entries beyond the list, then overflow lists (rare), by the bin's lane
#pragma unroll
            for (int j = 0; j < NBL; j++) {
                const int d = l + TL_PLANES * j;
                if (d >= 27) break;
                const int c = min(cntq[j], TL_BCAP);
                if (pos[j] + c > TL_PLIST) {
                    int e[TL_BCAP];
                    bucket_sorted(D, hq[j], c, e);
#pragma unroll
                    for (int k = 0; k < TL_BCAP; k++) {
                        if (k >= c || pos[j] + k < TL_PLIST) continue;
                        const float4* src = D.crec + (long long)e[k] * 3;
                        visit(src, src[0], src[1], d);
                    }
                }
                if (cntq[j] > TL_BCAP) {
                    // visited in increasing candidate number (= particle index)
                    unsigned long long e = D.htab[hq[j]];
                    if ((unsigned)(e >> 32) == gen) {
                        const int head = (int)(e & 0xFFFFFFFFull);
                        int last = -1;
                        while (true) {
                            int best = INT_MAX;
                            for (int q = head; q >= 0; q = D.hnext[q])
                                if (q > last && q < best) best = q;
                            if (best == INT_MAX) break;
                            const float4* src = D.crec + (long long)best * 3;
                            visit(src, src[0], src[1], d);
                            last = best;
                        }
                    }
                }
            }
        }
        // fixed-order sum over the lanes of the group
        for (int a = 0; a < 3; a++) {
            static_assert(TL_PLANES == 4 || TL_PLANES == 8, "the lane sum below covers 4 or 8 lanes");
            if constexpr (TL_PLANES == 8) Jt[a] += lane_xor<4>(Jt[a]);
            Jt[a] += lane_xor<2>(Jt[a]);
            Jt[a] += lane_xor<1>(Jt[a]);
        }
        __syncthreads();
        if (has && l == 0) {
            const int nn = s_nnew[sub];
            D.ph_n[(long long)hnew * N + p] = (stamp << 8) | (nn < TL_PCAP ? nn : TL_PCAP);
            D.Jmat[p] = Jt[0];
            D.Jmat[N + p] = Jt[1];
            D.Jmat[2 * N + p] = Jt[2];
        }
    }
}

#define TL_WRAP(NAME, PARAMS, ARGS)                                                                           \
    __global__ __launch_bounds__(256) void k_##NAME(SceneK S, SceneD D PARAMS)                              \
    {                                                                                                       \
        NAME##_body(S, D, blockIdx.x ARGS);                                                                 \
    }                                                                                                       \
    __global__ __launch_bounds__(256) void k_##NAME##_b(const SceneK* __restrict__ Ks,                       \
                                                        const SceneD* __restrict__ Ds,                       \
                                                        const int2* __restrict__ it PARAMS)                  \
    {                                                                                                       \
        const int2 t = it[blockIdx.x];                                                                      \
        NAME##_body(Ks[t.x], Ds[t.x], t.y ARGS);                                                            \
    }
#define TL_COMMA ,
TL_WRAP(cellmask, TL_COMMA int with_static TL_COMMA int force, TL_COMMA with_static TL_COMMA force)
// one workgroup per brick: the one-stream substeps of scenes of few bricks, and
// batches (whose small scenes have many bricks next to a code change: there one
// workgroup per work item measured faster than several)
TL_WRAP(cand, TL_COMMA int force, TL_COMMA force)
TL_WRAP(bin_insert, , )
__global__ __launch_bounds__(256) void k_bin_insert_scan(SceneK S, SceneD D) { bin_insert_body(S, D, blockIdx.x, 1); }
// at most 128 VGPRs: four waves per SIMD
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_pairs(SceneK S, SceneD D)
{
    pairs_body(S, D, blockIdx.x);
}
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_pairs_b(
    const SceneK* __restrict__ Ks, const SceneD* __restrict__ Ds, const int2* __restrict__ it)
{
    const int2 t = it[blockIdx.x];
    pairs_body(Ks[t.x], Ds[t.x], t.y);
}
// The slot-table pass and the pair search in one launch: the first nn blocks build
// slot tables (dispatched first: the pair blocks alone fill the chip, and stride over
// the candidates whenever they start), the others search pairs.  The two touch
// disjoint arrays (the slot pass reads the codes without the candidate bit), so they
// need no order; one launch replaces a second stream and the events that fork and
// join it.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_pairs_slots(SceneK S, SceneD D,
                                                                                           int nn, int dst, int src)
{
    if ((int)blockIdx.x < nn)
        slots_body(S, D, blockIdx.x, dst, src, 0);
    else
        pairs_body(S, D, blockIdx.x - nn);
}
__global__ __launch_bounds__(TL_SCAN_T) void k_cscan(SceneK S, SceneD D) { cscan_body(S, D, 0); }
__global__ __launch_bounds__(TL_SCAN_T) void k_cscan_b(const SceneK* __restrict__ Ks, const SceneD* __restrict__ Ds,
                                                       const int2* __restrict__ it)
{
    const int2 t = it[blockIdx.x];
    cscan_body(Ks[t.x], Ds[t.x], t.y);
}


template <class KP, class KB, class... Args>
static hipError_t tl_run_t(const TlLaunch& L, int kind, int plain_blocks, int threads, KP kp, KB kb, Args... args)
{
    if (L.S) {
        if (plain_blocks <= 0) return hipSuccess;
        hipLaunchKernelGGL(kp, dim3(plain_blocks), dim3(threads), 0, L.st, *L.S, *L.D, args...);
    } else {
        if (L.n_items[kind] <= 0) return hipSuccess;
        hipLaunchKernelGGL(kb, dim3(L.n_items[kind]), dim3(threads), 0, L.st, L.Ks, L.Ds, L.items[kind], args...);
    }
    return hipGetLastError();
}

template <class KP, class KB, class... Args>
static hipError_t tl_run(const TlLaunch& L, int kind, int plain_blocks, KP kp, KB kb, Args... args)
{
    return tl_run_t(L, kind, plain_blocks, 256, kp, kb, args...);
}

extern "C" {
hipError_t tl_launch_cellmask(const TlLaunch* L, int with_static, int force)
{
    int nb = 0;
    if (L->S) nb = (int)(((long long)L->S->cbx * L->S->cby * L->S->cbz * TL_CELLS + 255) / 256);
    return tl_run(*L, IT_CELL, nb, k_cellmask, k_cellmask_b, with_static, force);
}

// candidate bits and lists, then the global candidate offsets
hipError_t tl_launch_cand(const TlLaunch* L, int force)
{
    hipError_t e;
    if (L->S) { // one scene: TL_CBRICKS bricks per workgroup
        const int n = L->D->n_active;
        if (n > 0)
            hipLaunchKernelGGL(k_cand_multi, dim3((n + TL_CBRICKS - 1) / TL_CBRICKS), dim3(256), 0, L->st, *L->S,
                               *L->D, force);
        e = hipGetLastError();
    } else {
        e = tl_run(*L, IT_BRICK, 0, k_cand, k_cand_b, force);
    }
    if (e != hipSuccess) return e;
    return tl_run_t(*L, IT_SCENE, 1, TL_SCAN_T, k_cscan, k_cscan_b);
}

// one substep of pair search and impulses: binning, pairs
hipError_t tl_launch_contact(const TlLaunch* L)
{
    const int nbrick = L->S ? L->D->n_active : 0;
    if (L->S && nbrick == 0) return hipSuccess;
    hipError_t e = tl_run(*L, IT_BRICK, nbrick, k_bin_insert, k_bin_insert_b);
    if (e != hipSuccess) return e;
    return tl_run(*L, IT_PAIR, L->S ? L->S->pair_blocks : 0, k_pairs, k_pairs_b);
}

hipError_t tl_launch_slots(const TlLaunch* L, int dst, int src, int force);

// One scene of few bricks, substep with a label pass: candidates, binning with the
// candidate offsets summed per block (no scan launch), then pairs together with the
// slot tables dst (built from src).
hipError_t tl_launch_cand_contact_slots(const TlLaunch* L, int dst, int src)
{
    if (!L->S) return hipErrorInvalidValue;
    const int nbrick = L->D->n_active;
    if (nbrick == 0) return tl_launch_slots(L, dst, src, 0);
    const int np = L->S->pair_blocks;
    const int nn = (int)((L->S->NN + 255) / 256);
    hipLaunchKernelGGL(k_cand, dim3(nbrick), dim3(256), 0, L->st, *L->S, *L->D, 0);
    hipLaunchKernelGGL(k_bin_insert_scan, dim3(nbrick), dim3(256), 0, L->st, *L->S, *L->D);
    hipLaunchKernelGGL(k_pairs_slots, dim3(nn + np), dim3(256), 0, L->st, *L->S, *L->D, nn, dst, src);
    return hipGetLastError();
}
}
