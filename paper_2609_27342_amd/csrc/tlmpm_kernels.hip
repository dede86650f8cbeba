// tlmpm_kernels.hip -- gfx950 kernels of one TLMPM cutting substep.
//
// Work decomposition.  Particles are sorted into bricks of 4x4x4 reference cells;
// inside a brick by cell parity class (8 classes of 8 cells that share no grid node)
// and then by cell.  One 512-thread workgroup owns one brick: wave w holds parity
// class w, lane (i, j) holds particle j of cell i of that class, where the bits of
// j sit at lane bits 0, 1 and 4 and those of i at lane bits 2, 3 and 5 (a cell's 8
// lanes are two quads in rows 2q and 2q+1 of the wave).  A brick touches the 5x5x5
// box of nodes around it.
//
// Particle-to-grid sums are gathers with a fixed order, without float atomics:
//   1. every lane forms its particle's contribution to the 8 corner nodes of its
//      cell;
//   2. an 8-lane butterfly reduce-scatter leaves in lane (i, k) the sum of cell i's
//      particles for corner k (the j bit 2 stage swaps rows with
//      v_permlane16_swap, the other two add across the quad with DPP);
//   3. the 8 waves add their per-node sums into LDS one class after another;
//   4. the box sums are written as this brick's partial; a node's total is the sum
//      of the partials of the (up to 8) bricks around it, formed in fixed order by
//      the kernel that consumes it.
//
// Each node holds one slot (logical grid, Sec. III-D) per side code present in its
// 8 incident cells, in ascending code order; coupling (Eq. 8) is done per node when
// a box is finalized.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>

#include "tlmpm_common.h"
#include "tlmpm_band.h"
#include "tlmpm_reach.h"
#include "tlmpm_device.h"


DEV int box_index(int X, int Y, int Z) { return (Z * 5 + Y) * 5 + X; }

// Global node id of box node (X, Y, Z) of cell brick (bx, by, bz); -1 outside the grid.
DEV long long box_gid(const SceneK& S, int bx, int by, int bz, int X, int Y, int Z)
{
    int gx = bx * TL_B + X, gy = by * TL_B + Y, gz = bz * TL_B + Z;
    if (gx > S.cx || gy > S.cy || gz > S.cz) return -1;
    long long nb = ((long long)(gz >> 2) * S.nby + (gy >> 2)) * S.nbx + (gx >> 2);
    return (nb << 6) | ((gz & 3) * 16 + (gy & 3) * 4 + (gx & 3));
}

// ------------------------------------------------------------------- box slot table
struct BoxTab {
    int cnt[TL_BOXN];
    int base[TL_BOXN + 1];
    long long gid[TL_BOXN];
    uint32_t code[TL_BOX_SLOTS];
    unsigned char node_of[TL_BOX_SLOTS];
};

// Phase 1: slot counts of the 125 box nodes (threads < 125, no barrier).
DEV void box_counts(const SceneK& S, const uint8_t* cnt, int bx, int by, int bz, BoxTab& T)
{
    const int tid = threadIdx.x;
    if (tid < TL_BOXN) {
        int X = tid % 5, Y = (tid / 5) % 5, Z = tid / 25;
        long long g = box_gid(S, bx, by, bz, X, Y, Z);
        T.gid[tid] = g;
        T.cnt[tid] = g >= 0 ? (int)cnt[g] : 0;
    }
}

// Phase 2 (after a barrier): exclusive scan of the counts by wave `wave`.
DEV void box_scan(BoxTab& T, int* s_total, int wave)
{
    const int tid = threadIdx.x;
    if ((tid >> 6) != wave) return;
    const int l = tid & 63;
    int a = 2 * l, b = 2 * l + 1;
    int va = a < TL_BOXN ? T.cnt[a] : 0;
    int vb = b < TL_BOXN ? T.cnt[b] : 0;
    int sum = va + vb, incl = sum;
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(incl, o, 64);
        if (l >= o) incl += t;
    }
    int excl = incl - sum;
    if (a < TL_BOXN) T.base[a] = excl;
    if (b < TL_BOXN) T.base[b] = excl + va;
    if (l == 63) {
        T.base[TL_BOXN] = incl;
        *s_total = incl;
    }
}

// Phase 3 (after a barrier, threads < 125): codes of this thread's node.
// The same in two steps, so that the code loads are in flight together with the
// loads that follow (the partial gather): the first two codes of node bn into
// registers, then into the table (further codes loaded there).
DEV void codes_pre(const SceneK& S, const uint32_t* scode, const BoxTab& T, int bn, uint32_t pre[2])
{
    const int c = T.cnt[bn];
    const long long g = T.gid[bn];
    pre[0] = c > 0 ? scode[g] : 0u;
    pre[1] = c > 1 ? scode[S.NN + g] : 0u;
}

DEV void codes_put(const SceneK& S, const uint32_t* scode, BoxTab& T, int bn, const uint32_t pre[2])
{
    const int c = T.cnt[bn], b0 = T.base[bn];
    const long long g = T.gid[bn];
    for (int s = 0; s < c; s++) {
        T.code[b0 + s] = s == 0 ? pre[0] : s == 1 ? pre[1] : scode[(long long)s * S.NN + g];
        T.node_of[b0 + s] = (unsigned char)bn;
    }
}

DEV int find_slot(const BoxTab& T, int bn, uint32_t key)
{
    int c = T.cnt[bn], b0 = T.base[bn];
    if (c == 1) return T.code[b0] == key ? b0 : -1;
    for (int s = 0; s < c; s++)
        if (T.code[b0 + s] == key) return b0 + s;
    return -1;
}

// Partial arrays hold every active brick's sums over its 5x5x5 box of nodes:
// [active brick][slot][box node][QP floats], the Q components of one node-slot
// contiguous (QP = Q rounded up to 4 floats).  A node's slot index is global (the
// node's slot table), so all bricks that share the node use the same slot.
template <int Q>
struct QPad {
    static constexpr int value = (Q + 3) & ~3;
};

// Active indices of the 27 bricks around (bx, by, bz) (-1: none), by threads
// [TL_BOXN, TL_BOXN + 27) of the block; read after the next barrier.
DEV void load_neighbours(const SceneK& S, const SceneD& D, int bx, int by, int bz, int* nb)
{
    const int t = (int)threadIdx.x - TL_BOXN;
    if (t < 0 || t >= 27) return;
    const int x = bx + t % 3 - 1, y = by + (t / 3) % 3 - 1, z = bz + t / 9 - 1;
    nb[t] = (x < 0 || y < 0 || z < 0 || x >= S.cbx || y >= S.cby || z >= S.cbz)
                ? -1
                : D.bact[((long long)z * S.cby + y) * S.cbx + x];
}

// Sums of all slots of box node bn over the bricks that contributed to it, written
// to dst[slot * Q + c], formed by the 4 threads u = 0..3 of a quad (lanes 4 bn ..
// 4 bn + 3): contributor d is the brick at home - (d & 1, d >> 1 & 1, d >> 2 & 1),
// which holds the node at box position (l + 4 * offset); thread u loads contributors u
// and u + 4 (each its first partial plus, where xflag is set, the partial of its later
// same-code rounds), the quad adds its 4 sums ((0 + 1) + (2 + 3)) and thread 0
// writes them.  The order is fixed: results are bitwise reproducible.
template <int Q>
DEV void gather_node4(const SceneK& S, const int* nb, const float* __restrict__ part, const float* __restrict__ xpart,
                      const int* __restrict__ xflag, const BoxTab& T, int bn, int u, float* dst)
{
    constexpr int QP = QPad<Q>::value;
    const int c = T.cnt[bn], b0 = T.base[bn];
    const int X = bn % 5, Y = (bn / 5) % 5, Z = bn / 25;
    const int lx = X & 3, ly = Y & 3, lz = Z & 3;
    unsigned cbase[2] = {0u, 0u};
    unsigned valid = 0, extra = 0;
#pragma unroll
    for (int e = 0; e < 2; e++) {
        const int d = u + 4 * e;
        const int dx = d & 1, dy = (d >> 1) & 1, dz = (d >> 2) & 1;
        if ((dx && lx) || (dy && ly) || (dz && lz)) continue;
        const int ai = nb[((Z >> 2) - dz + 1) * 9 + ((Y >> 2) - dy + 1) * 3 + ((X >> 2) - dx + 1)];
        if (ai < 0) continue;
        const int pn = (lx + 4 * dx) + 5 * (ly + 4 * dy) + 25 * (lz + 4 * dz);
        cbase[e] = (unsigned)ai * (unsigned)(S.scap * TL_BOXN) + (unsigned)pn;
        valid |= 1u << e;
        if (xflag && xflag[ai]) extra |= 1u << e;
    }
    for (int s = 0; s < c; s++) {
        float acc[QP];
#pragma unroll
        for (int q = 0; q < QP; q++) acc[q] = 0.0f;
#pragma unroll
        for (int e = 0; e < 2; e++) {
            if (!(valid & (1u << e))) continue;
            const size_t rec = (size_t)(cbase[e] + (unsigned)(s * TL_BOXN)) * QP;
            const float4* pp = (const float4*)(part + rec);
            float4 v4[QP / 4];
#pragma unroll
            for (int q4 = 0; q4 < QP / 4; q4++) v4[q4] = pp[q4];
            if (extra & (1u << e)) {
                const float4* xp = (const float4*)(xpart + rec);
#pragma unroll
                for (int q4 = 0; q4 < QP / 4; q4++) {
                    const float4 x4 = xp[q4];
                    v4[q4].x += x4.x;
                    v4[q4].y += x4.y;
                    v4[q4].z += x4.z;
                    v4[q4].w += x4.w;
                }
            }
#pragma unroll
            for (int q4 = 0; q4 < QP / 4; q4++) {
                acc[4 * q4 + 0] += v4[q4].x;
                acc[4 * q4 + 1] += v4[q4].y;
                acc[4 * q4 + 2] += v4[q4].z;
                acc[4 * q4 + 3] += v4[q4].w;
            }
        }
#pragma unroll
        for (int q = 0; q < Q; q++) {
            acc[q] += lane_xor<1>(acc[q]);
            acc[q] += lane_xor<2>(acc[q]);
        }
        if (u == 0)
#pragma unroll
            for (int q = 0; q < Q; q++) dst[(b0 + s) * Q + q] = acc[q];
    }
}

// Compatibility coupling of one 3-vector field at a node with slots [b0, b0+c)
// (Eq. 8): f_a += (1/M) sum_{b != a, compatible} (m_a f_b - m_b f_a), M = sum of
// all slot masses; fields read from src (stride Q, offset off) and written to dst
// (stride 3), all pre-exchange values.
template <int Q>
DEV void couple_node(const BoxTab& T, int b0, int c, const float* src, int off, float* dst)
{
    if (c == 1) {
        for (int j = 0; j < 3; j++) dst[b0 * 3 + j] = src[b0 * Q + off + j];
        return;
    }
    float M = 0.0f;
    for (int a = 0; a < c; a++) M += src[(b0 + a) * Q];
    float invM = M > 0.0f ? 1.0f / M : 0.0f;
    for (int a = 0; a < c; a++) {
        uint32_t ca = T.code[b0 + a];
        float ma = src[(b0 + a) * Q];
        float fa[3] = {src[(b0 + a) * Q + off], src[(b0 + a) * Q + off + 1], src[(b0 + a) * Q + off + 2]};
        float acc[3] = {0.0f, 0.0f, 0.0f};
        for (int b = 0; b < c; b++) {
            if (b == a || codes_conflict(ca, T.code[b0 + b])) continue;
            float mb = src[(b0 + b) * Q];
            for (int j = 0; j < 3; j++) acc[j] += ma * src[(b0 + b) * Q + off + j] - mb * fa[j];
        }
        for (int j = 0; j < 3; j++) dst[(b0 + a) * 3 + j] = fa[j] + acc[j] * invM;
    }
}

// ------------------------------------------------------------- particle geometry
struct Lane {
    int w, lane, i, j;
    int cxl, cyl, czl; // cell inside the brick
    int beg, count;    // particles of the cell
};

DEV Lane lane_of(const SceneD& D, int brick)
{
    Lane L;
    int tid = threadIdx.x;
    L.w = tid >> 6;
    L.lane = tid & 63;
    L.i = ((L.lane >> 2) & 3) | ((L.lane >> 3) & 4); // lane bits 2, 3, 5
    L.j = (L.lane & 3) | ((L.lane >> 2) & 4);        // lane bits 0, 1, 4
    L.cxl = 2 * (L.i & 1) + (L.w & 1);
    L.cyl = 2 * ((L.i >> 1) & 1) + ((L.w >> 1) & 1);
    L.czl = 2 * ((L.i >> 2) & 1) + ((L.w >> 2) & 1);
    const int* cs = D.cell_start + (long long)brick * TL_CELLS + L.w * 8 + L.i;
    L.beg = cs[0];
    L.count = cs[1] - cs[0];
    return L;
}

// Particle of this lane in round r.  Bricks whose cells each hold one code take
// particle 8 r + j of the lane's cell; bricks with a mixed cell take particle j of
// the cell's r-th same-code group (group table built when the codes change).
DEV bool lane_particle(const SceneD& D, int bi, bool grouped, const Lane& L, int r, long long& p)
{
    if (!grouped) {
        const int jj = 8 * r + L.j;
        p = L.beg + (jj < L.count ? jj : 0);
        return jj < L.count;
    }
    p = L.beg;
    if (r >= TL_GMAX) return false;
    const int m = D.gmeta[((long long)bi * TL_CELLS + L.w * 8 + L.i) * TL_GMAX + r];
    const int cnt = m & 15, off = m >> 4;
    if (L.j >= cnt) return false;
    p = D.gperm[L.beg + off + L.j];
    return true;
}

// fractional position inside the base cell (reading R1), in [0, 1]
DEV void frac_of(const SceneK& S, const float* X, int gxc, int gyc, int gzc, float t[3])
{
    double q0 = ((double)X[0] - S.ox) * S.inv_dx_d - (double)gxc;
    double q1 = ((double)X[1] - S.oy) * S.inv_dx_d - (double)gyc;
    double q2 = ((double)X[2] - S.oz) * S.inv_dx_d - (double)gzc;
    t[0] = fminf(fmaxf((float)q0, 0.0f), 1.0f);
    t[1] = fminf(fmaxf((float)q1, 0.0f), 1.0f);
    t[2] = fminf(fmaxf((float)q2, 0.0f), 1.0f);
}

DEV void corner_weights(const float t[3], int k, float& wx, float& wy, float& wz)
{
    wx = (k & 1) ? t[0] : 1.0f - t[0];
    wy = (k & 2) ? t[1] : 1.0f - t[1];
    wz = (k & 4) ? t[2] : 1.0f - t[2];
}

// --------------------------------------------------------- butterfly reduce-scatter
// Weights of the 8 corners of a lane's cell in the order the relative butterfly
// takes them: corner r has x bit (r & 1) and y bit (r >> 1 & 1) relative to the
// lane's own corner j (clear: j's side, set: the other side) and z bit (r >> 2)
// absolute, so its absolute index is r ^ (j & 3).  Each factor is the one
// corner_weights gives for the absolute corner.
struct CornerW {
    float wx[2], wy[2], wz[2];
};

DEV CornerW corner_table(const float t[3], int j)
{
    CornerW c;
    const bool bx = j & 1, by = (j >> 1) & 1;
    const float ox = 1.0f - t[0], oy = 1.0f - t[1];
    c.wx[0] = bx ? t[0] : ox;
    c.wx[1] = bx ? ox : t[0];
    c.wy[0] = by ? t[1] : oy;
    c.wy[1] = by ? oy : t[1];
    c.wz[0] = 1.0f - t[2];
    c.wz[1] = t[2];
    return c;
}

// gen(r, out) produces this lane's contribution to corner r of its cell.  Result:
// res[Q] = sum over the 8 lanes of the cell group of their values for corner j (the
// lane's own).  REL: corners in the order of CornerW (x and y bits relative to j);
// else absolute corner indices.  Stage 1 pairs j with j ^ 4 (lane ^ 16):
// v_permlane16_swap of (z = 0, z = 1) leaves in the even row (z bit of j clear) its
// own and its partner's z = 0 values, in the odd row the z = 1 values; stages 2 and
// 3 pair j ^ 2 and j ^ 1 within the quad, each lane sending the value of the
// partner's side (REL: its other-side value, no select).  The sum tree is ((j,
// j^4), (j^2, j^6)), ((j^1, j^5), (j^3, j^7)), own operand first, for every lane
// order.  Corners are generated in (z = 0, z = 1) pairs, so at most 4 x Q partial
// sums are live.
template <int Q, bool REL, class Gen>
DEV void reduce_scatter8(Gen&& gen, float (&res)[Q], int j)
{
    float c1[4][Q];
#pragma unroll
    for (int rr = 0; rr < 4; rr++) {
        float lo[Q], hi[Q];
        gen(rr, lo);
        gen(rr | 4, hi);
#pragma unroll
        for (int q = 0; q < Q; q++) {
            const auto sw = __builtin_amdgcn_permlane16_swap(__float_as_uint(lo[q]), __float_as_uint(hi[q]), false,
                                                             false);
            c1[rr][q] = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
        }
    }
    float c2[2][Q];
    const bool b1 = (j >> 1) & 1;
#pragma unroll
    for (int rr = 0; rr < 2; rr++)
#pragma unroll
        for (int q = 0; q < Q; q++) {
            if constexpr (REL) {
                c2[rr][q] = c1[rr][q] + lane_xor<2>(c1[rr | 2][q]);
            } else {
                const float send = b1 ? c1[rr][q] : c1[rr | 2][q];
                const float keep = b1 ? c1[rr | 2][q] : c1[rr][q];
                c2[rr][q] = keep + lane_xor<2>(send);
            }
        }
    const bool b0 = j & 1;
#pragma unroll
    for (int q = 0; q < Q; q++) {
        if constexpr (REL) {
            res[q] = c2[0][q] + lane_xor<1>(c2[1][q]);
        } else {
            const float send = b0 ? c2[0][q] : c2[1][q];
            const float keep = b0 ? c2[1][q] : c2[0][q];
            res[q] = keep + lane_xor<1>(send);
        }
    }
}

// Adds a wave's per-node sums to the LDS box accumulator, one parity class after
// another (fixed order).  The QA + QB components come from two generators (two
// butterflies keep fewer partial sums live).  Every 8-lane group holds particles
// of one code (bricks with a mixed cell are processed in same-code groups).
// Component q of the generated values is stored at (q + ROT) mod Q of a slot.
template <int QA, int QB, bool REL, int ROT = 0, class GA, class GB>
DEV void accumulate_classes(const Lane& L, bool valid, uint32_t key, GA&& ga, GB&& gb, const BoxTab& T, float* acc,
                            int* status)
{
    constexpr int Q = QA + QB;
    const int leader = L.lane & ~0x13; // j = 0 of the lane's cell
    const uint32_t lkey = __shfl(key, leader, 64);
    const bool gvalid = __shfl((int)valid, leader, 64) != 0;
    if (__any(valid && key != lkey) && L.lane == 0) atomicOr(status, TL_ST_LOOKUP);
    float res[Q];
    {
        float ra[QA];
        reduce_scatter8<QA, REL>(ga, ra, L.j);
#pragma unroll
        for (int q = 0; q < QA; q++) res[q] = ra[q];
        if constexpr (QB > 0) {
            float rb[QB];
            reduce_scatter8<QB, REL>(gb, rb, L.j);
#pragma unroll
            for (int q = 0; q < QB; q++) res[QA + q] = rb[q];
        }
    }
    const int bn = box_index(L.cxl + (L.j & 1), L.cyl + ((L.j >> 1) & 1), L.czl + ((L.j >> 2) & 1));
    for (int phase = 0; phase < 8; phase++) {
        lds_barrier();
        if (L.w != phase || !gvalid) continue;
        int sl = find_slot(T, bn, lkey);
        if (sl < 0)
            atomicOr(status, TL_ST_LOOKUP);
        else
#pragma unroll
            for (int q = 0; q < Q; q++) acc[sl * Q + (q + ROT) % Q] += res[q];
    }
    lds_barrier();
}

// Writes the box accumulator as this brick's partial (layout of gather_node4).
template <int Q>
DEV void write_partials(const SceneK& S, float* __restrict__ part, int bi, const BoxTab& T, int total, const float* acc)
{
    constexpr int QP = QPad<Q>::value;
    for (int q = threadIdx.x; q < total; q += blockDim.x) {
        int bn = T.node_of[q];
        int s = q - T.base[bn];
        float4* pp = (float4*)(part + (((long long)bi * S.scap + s) * TL_BOXN + bn) * QP);
        float v[QP];
#pragma unroll
        for (int c = 0; c < QP; c++) v[c] = c < Q ? acc[q * Q + c] : 0.0f;
#pragma unroll
        for (int q4 = 0; q4 < QP / 4; q4++) pp[q4] = make_float4(v[4 * q4], v[4 * q4 + 1], v[4 * q4 + 2], v[4 * q4 + 3]);
    }
}

// ------------------------------------------------------- history-based friction
// Tangential spring transported to the current tangent plane (length kept), trial
// force -k_t u - c_t v_t, stick below mu_s f_n, else slip at mu_d f_n with the
// spring reset to match the applied force (Eq. 12).
DEV void friction(const SceneK& S, const float vrel[3], const float n[3], float fn, float meff, float u[3],
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

// One rigid body against one particle (Eqs. 14-16, 5).  body 0 = floor, else tool.
// Returns the impulse on the particle in J (added), updates D and the wrench sums.
// The contact geometry (closest point, gap, normal, front-band coordinates) is
// formed in FP64 from the exact current position x = X + u: the normal impulse is
// s_n m / dt times the gap, and for a particle close to the zero-thickness blade
// the normal is (x - x_c) / |x - x_c| of a short vector, so FP32 rounding of the
// positions (1e-8 m at 0.2 m) would shift the gap and turn the normal by far more
// than the FP32 state error.
DEV void rigid_one(const SceneK& S, const SceneD& D, const DevTool* T, int slot, long long p, const double x[3],
                   const float v[3], float m, float V0, float R, int stamp, double jdt, float J[3], float& Dp,
                   float Dstart, float* wr)
{
    const float dt = S.dt;
    double adv = (T && (T->flags & TL_TOOL_ADVANCE)) ? jdt : 0.0;
    float nB[3], phi, vB[3] = {0.0f, 0.0f, 0.0f}, arm[3] = {0.0f, 0.0f, 0.0f};
    float invm = 0.0f;
    double r[3] = {0.0, 0.0, 0.0}; // x - x_e of a tool
    if (!T) {
        nB[0] = 0.0f;
        nB[1] = 0.0f;
        nB[2] = 1.0f;
        phi = (float)((x[2] - (double)S.floor_z) - (double)R);
    } else {
        const DevBlade& B = T->b;
        for (int a = 0; a < 3; a++) r[a] = x[a] - (B.xe[a] + adv * B.ve[a]);
        double al = r[0] * B.e[0] + r[1] * B.e[1] + r[2] * B.e[2];
        double be = -(r[0] * B.d[0] + r[1] * B.d[1] + r[2] * B.d[2]);
        al = fmin(fmax(al, -B.half_len), B.half_len);
        be = fmin(fmax(be, 0.0), B.b_back);
        double df[3];
        for (int a = 0; a < 3; a++) df[a] = r[a] - al * B.e[a] + be * B.d[a]; // x - x_c
        const double dist = sqrt(df[0] * df[0] + df[1] * df[1] + df[2] * df[2]);
        if (dist > 0.0)
            for (int a = 0; a < 3; a++) nB[a] = (float)(df[a] / dist);
        else
            for (int a = 0; a < 3; a++) nB[a] = (float)B.n[a];
        phi = (float)(dist - (double)R);
        for (int a = 0; a < 3; a++)
            arm[a] = (float)((x[a] - df[a]) - (T->xB[a] + adv * T->vB[a])); // x_c - x_B
        float wxr[3] = {T->wB[1] * arm[2] - T->wB[2] * arm[1], T->wB[2] * arm[0] - T->wB[0] * arm[2],
                        T->wB[0] * arm[1] - T->wB[1] * arm[0]};
        for (int a = 0; a < 3; a++) vB[a] = (float)T->vB[a] + wxr[a];
        // inverse effective mass of the tool at xc along nB: w_B + 1/M + (r x n) . I^-1 (r x n)
        const float cr[3] = {arm[1] * nB[2] - arm[2] * nB[1], arm[2] * nB[0] - arm[0] * nB[2],
                             arm[0] * nB[1] - arm[1] * nB[0]};
        float ang = 0.0f;
        for (int a = 0; a < 3; a++)
            ang += cr[a] * (T->iinv[3 * a] * cr[0] + T->iinv[3 * a + 1] * cr[1] + T->iinv[3 * a + 2] * cr[2]);
        invm = T->invm + T->imass + ang;
    }
    float vrel[3] = {v[0] - vB[0], v[1] - vB[1], v[2] - vB[2]};
    float vrn = vrel[0] * nB[0] + vrel[1] * nB[1] + vrel[2] * nB[2];
    float phihat = phi + dt * fminf(vrn, 0.0f);
    float meff = 1.0f / (1.0f / m + invm);
    float Jn = S.s_n * meff / dt * fmaxf(-phihat, 0.0f);
    if (!(Jn > 0.0f)) return;
    float* h = D.hist + (long long)slot * 4 * S.N;
    float u[3] = {0.0f, 0.0f, 0.0f};
    if (__float_as_int(h[3 * S.N + p]) == stamp - 1) {
        u[0] = h[p];
        u[1] = h[S.N + p];
        u[2] = h[2 * S.N + p];
    }
    float ft[3];
    friction(S, vrel, nB, Jn / dt, meff, u, ft);
    h[p] = u[0];
    h[S.N + p] = u[1];
    h[2 * S.N + p] = u[2];
    h[3 * S.N + p] = __int_as_float(stamp);
    float JpB[3] = {Jn * nB[0] + ft[0] * dt, Jn * nB[1] + ft[1] * dt, Jn * nB[2] + ft[2] * dt};
    if (T && (T->flags & TL_TOOL_CUTTING)) {
        const DevBlade& B = T->b;
        const double sv = r[0] * B.n[0] + r[1] * B.n[1] + r[2] * B.n[2];
        const double lv = r[0] * B.e[0] + r[1] * B.e[1] + r[2] * B.e[2];
        const double fv = r[0] * B.d[0] + r[1] * B.d[1] + r[2] * B.d[2];
        float uc = ((float)B.ve[0] - v[0]) * (float)B.d[0] + ((float)B.ve[1] - v[1]) * (float)B.d[1] +
                   ((float)B.ve[2] - v[2]) * (float)B.d[2];
        if (fabs(sv) <= B.half_width && fabs(lv) <= B.half_len && fv >= 0.0 && fv <= B.b_lead && uc > S.u_min) {
            float dd[3] = {(float)B.d[0], (float)B.d[1], (float)B.d[2]};
            float Jc = fmaxf(JpB[0] * dd[0] + JpB[1] * dd[1] + JpB[2] * dd[2], 0.0f);
            if (Dstart < 1.0f) {
                float Wth = S.G_c * powf(V0, 2.0f / 3.0f) * (1.0f - S.zeta) / S.zeta;
                Dp = fminf(Dp + Jc * uc / Wth, 1.0f);
            } else {
                for (int a = 0; a < 3; a++) JpB[a] -= Jc * dd[a];
            }
        }
    }
    for (int a = 0; a < 3; a++) J[a] += JpB[a];
    if (wr) {
        float Fb[3] = {-JpB[0] / dt, -JpB[1] / dt, -JpB[2] / dt};
        wr[0] += Fb[0];
        wr[1] += Fb[1];
        wr[2] += Fb[2];
        wr[3] += arm[1] * Fb[2] - arm[2] * Fb[1];
        wr[4] += arm[2] * Fb[0] - arm[0] * Fb[2];
        wr[5] += arm[0] * Fb[1] - arm[1] * Fb[0];
    }
}

// --------------------------------------------------------------------------- K_A
// P2G kernel (one brick per workgroup).  If f_pending: finalize the remapped
// velocities of the previous substep's MUSL re-scatter on the box (tables rs),
// apply the deformation-gradient update and write F.  Then, if do_p2g: stress,
// tool/floor contact, and the label-masked P2G of (m, p, dp) (Eq. 2 with external
// and contact impulses, Eqs. 13, 16) into this brick's partials (tables cur).
struct KA_Args {
    int do_p2g;      // 0: only the pending F update
    int tabs_differ; // cur != rsb (applies to scenes with a pending F update)
    int cur;         // current slot table buffer
    int rsb;         // slot table buffer of the pending re-scatter
};

// --------------------------------------------------------------------- rigid contact
// Floor and tool contact of every particle of bricks whose AABB can reach a rigid
// body this substep (Eqs. 14-16, 5): impulses to Jrig, cutting progress D, contact
// springs, and per-brick wrench sums added to those of the call (wave tree, then
// waves in order).
DEV void rigid_body(const SceneK& S, const SceneD& D, int bi)
{
    if (!S.floor_on && !D.tinfo[1]) return; // no rigid body touches this scene
    const int n_tools = D.tinfo[0];
    const int stamp = D.ctr[0];
    const double jdt = (double)D.ctr[2] * S.dt_d; // substep of the call (TL_TOOL_ADVANCE poses)
    __shared__ int s_near[TL_MAX_TOOLS + 1];
    __shared__ int s_any;
    __shared__ float s_wr[4][TL_MAX_TOOLS * 6];
    const int brick = D.active[bi];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const long long N = S.N;
    if (tid <= TL_MAX_TOOLS) {
        float bb[7];
        brick_aabb(S, D, bi, brick, bb);
        int nr = 0;
        if (tid == 0)
            nr = S.floor_on ? brick_near_floor(bb, S.floor_z, S.Rmax, S.dt) : 0;
        else if (tid - 1 < n_tools)
            nr = (D.tools[tid - 1].flags & TL_TOOL_CONTACT) ? brick_near_tool(bb, D.tools[tid - 1], S.Rmax, S.dt, jdt)
                                                             : 0;
        s_near[tid] = nr;
    }
    if (lane < TL_MAX_TOOLS * 6) s_wr[wv][lane] = 0.0f;
    __syncthreads();
    if (tid == 0) {
        int any = 0;
        for (int b = 0; b <= n_tools; b++) any |= s_near[b];
        s_any = any;
        D.brig[brick] = any;
    }
    __syncthreads();
    const bool want_wrench = D.tinfo[1] != 0;
    if (s_any) {
        const int beg = D.cell_start[(long long)brick * TL_CELLS], end = D.cell_start[(long long)(brick + 1) * TL_CELLS];
        for (int p0 = beg; p0 < end; p0 += blockDim.x) {
            const int p = p0 + tid;
            const bool valid = p < end;
            double x[3] = {0.0, 0.0, 0.0};
            float v[3] = {0.0f, 0.0f, 0.0f}, m = 0.0f, V0 = 0.0f, R = 0.0f, Dp = 0.0f;
            float Jc[3] = {0.0f, 0.0f, 0.0f};
            if (valid) {
                for (int a = 0; a < 3; a++) {
                    x[a] = (double)D.X[a * N + p] + (double)D.u[a * N + p];
                    v[a] = D.v[a * N + p];
                }
                m = S.m_uniform ? S.m0 : D.m[p];
                V0 = S.v_uniform ? S.V0 : D.V0[p];
                R = 0.5f * S.s_R * cbrtf(V0);
                Dp = D.D[p];
                if (s_near[0]) rigid_one(S, D, nullptr, 0, p, x, v, m, V0, R, stamp, jdt, Jc, Dp, Dp, nullptr);
            }
            const float Ds = valid ? D.D[p] : 0.0f;
            for (int b = 0; b < n_tools; b++) {
                if (!s_near[b + 1]) continue;
                float wr[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
                if (valid) rigid_one(S, D, &D.tools[b], 1 + b, p, x, v, m, V0, R, stamp, jdt, Jc, Dp, Ds, wr);
                bool nz = wr[0] != 0.0f || wr[1] != 0.0f || wr[2] != 0.0f;
                if (want_wrench && __any(nz)) {
                    for (int q = 0; q < 6; q++) {
                        float val = wr[q];
                        for (int o = 32; o >= 1; o >>= 1) val += __shfl_xor(val, o, 64);
                        if (lane == 0) s_wr[wv][b * 6 + q] += val;
                    }
                }
            }
            if (valid) {
                D.Jrig[p] = Jc[0];
                D.Jrig[N + p] = Jc[1];
                D.Jrig[2 * N + p] = Jc[2];
                if (Dp != Ds) D.D[p] = Dp;
            }
        }
    }
    if (want_wrench && s_any) { // other bricks add nothing to the call's sums
        __syncthreads();
        if (tid < n_tools * 6) {
            float acc = 0.0f;
            for (int w = 0; w < 4; w++) acc += s_wr[w][tid];
            D.wpart[(long long)tid * D.n_active + bi] += (double)acc;
        }
    }
}

// MAT 0: Neo-Hookean only; MAT 1: the scene's material (Neo-Hookean or
// fixed-corotated) with Newtonian viscosity.
// part 0 takes the brick's first same-code round (all rounds unless the brick is
// split), part 1 the later rounds of a split brick (a brick whose cells hold two
// codes and need more than one round): the two run as separate workgroups, each
// with its own box partial, so that such bricks do not lengthen the launch.
template <int MAT, bool SPLIT>
DEV void p2g_body(const SceneK& S, const SceneD& D, int bi, KA_Args A, int part)
{
    __shared__ BoxTab Tc;
    __shared__ BoxTab Tr;
    __shared__ float s_vt[TL_BOX_SLOTS * 3];
    __shared__ float s_rsum[TL_BOX_SLOTS * 4];
    __shared__ float s_acc[TL_BOX_SLOTS * 7];
    __shared__ int s_total_r, s_total_c;
    __shared__ int s_nb[27];
    __shared__ int s_rounds;

    const int nround = SPLIT ? D.bround[bi] : 0; // rounds of a brick with a mixed cell, else 0
    if (SPLIT && part == 1 && nround <= 1) return;
    const int brick = D.active[bi];
    const bool grouped = D.bmixed[brick] != 0; // a cell holds two codes: same-code groups
    // (all mixed bricks split, or none: the decision does not depend on list order)
    const bool split = SPLIT && grouped && nround > 1 && S.xcap > 0 && D.ctr[3] <= S.xcap;
    const int r0 = part; // first round of this workgroup
    const int bx = brick % S.cbx, by = (brick / S.cbx) % S.cby, bz = brick / (S.cbx * S.cby);
    const int tid = threadIdx.x;
    const long long N = S.N;
    const float dt = S.dt;
    const bool fp = D.ctr[1] != 0;                              // F update of the last substep pending
    const bool use_r = fp;                                            // finalize v~ (tables rs)
    const bool use_c = A.do_p2g && ((A.tabs_differ && fp) || !fp); // separate P2G tables
    const bool xg_rs = SPLIT && D.xg[0] != 0; // the last G2P split bricks: their second re-scatter sums

    // ---- phase 1: cell index, box counts, brick-vs-tool tests, round-0 particle loads
    Lane L = lane_of(D, brick);
    if (use_r) box_counts(S, D.cnt[A.rsb], bx, by, bz, Tr);
    if (use_r) load_neighbours(S, D, bx, by, bz, s_nb);
    if (use_c) box_counts(S, D.cnt[A.cur], bx, by, bz, Tc);
    if (tid == 0) s_rounds = 0;
    // floor/tool impulses were computed for this brick by k_rigid
    const bool rig = A.do_p2g && (S.floor_on || D.tinfo[1]) && D.brig[brick] != 0;
    const int gxc = bx * TL_B + L.cxl, gyc = by * TL_B + L.cyl, gzc = bz * TL_B + L.czl;
    long long p = L.beg;
    bool valid = lane_particle(D, bi, grouped, L, r0, p);
    float Xp[3] = {0.0f, 0.0f, 0.0f}, H[9], vel[3] = {0.0f, 0.0f, 0.0f};
    uint32_t code = 0;
    auto load_particle = [&]() {
        Xp[0] = D.X[p];
        Xp[1] = D.X[N + p];
        Xp[2] = D.X[2 * N + p];
        code = D.code[p];
#pragma unroll
        for (int a = 0; a < 9; a++) H[a] = D.H[a * N + p];
        if (A.do_p2g)
            for (int a = 0; a < 3; a++) vel[a] = D.v[a * N + p];
    };
    if (valid) load_particle();
    lds_barrier();
    if (grouped) {
        if (tid == 0) s_rounds = D.bround[bi];
    } else if (L.j == 0) {
        atomicMax(&s_rounds, (L.count + 7) >> 3);
    }
    if (use_r) box_scan(Tr, &s_total_r, 0);
    if (use_c) box_scan(Tc, &s_total_c, 1);
    lds_barrier();
    const int total_r = use_r ? s_total_r : 0;
    const int total_c = use_c ? s_total_c : total_r;
    if (total_r > TL_BOX_SLOTS || total_c > TL_BOX_SLOTS) {
        if (tid == 0) atomicOr(D.status, TL_ST_BOX);
        return;
    }
    // ---- phase 3: per box node: codes, re-scatter sums, coupling, v~ (Eq. 8, MUSL)
    // (4 threads per node: the quad of lanes 4 bn .. 4 bn + 3)
    if ((tid >> 2) < TL_BOXN) {
        const int bn = tid >> 2, u = tid & 3;
        uint32_t pre_r[2], pre_c[2];
        if (u == 0 && use_r) codes_pre(S, D.scode[A.rsb], Tr, bn, pre_r);
        if (u == 0 && use_c) codes_pre(S, D.scode[A.cur], Tc, bn, pre_c);
        if (use_r) {
            const int c = Tr.cnt[bn], b0 = Tr.base[bn];
            if (c > 0) gather_node4<4>(S, s_nb, D.rs, D.rs_x, xg_rs ? D.xrs : nullptr, Tr, bn, u, s_rsum);
            if (u == 0) codes_put(S, D.scode[A.rsb], Tr, bn, pre_r);
            if (u == 0 && c > 0) {
                couple_node<4>(Tr, b0, c, s_rsum, 1, s_vt);
                for (int a = 0; a < c; a++) {
                    float m = s_rsum[(b0 + a) * 4];
                    float im = m > 0.0f ? 1.0f / m : 0.0f;
                    for (int jj = 0; jj < 3; jj++) s_vt[(b0 + a) * 3 + jj] *= im;
                }
            }
        }
        if (u == 0 && use_c) codes_put(S, D.scode[A.cur], Tc, bn, pre_c);
    }
    if (A.do_p2g)
        for (int q = tid; q < total_c * 7; q += TL_WG) s_acc[q] = 0.0f;
    lds_barrier();
    const BoxTab& T = use_c ? Tc : Tr;
    const int rounds = (split && part == 0) ? 1 : s_rounds;

    for (int r = r0; r < rounds; r++) {
        if (r > r0) {
            valid = lane_particle(D, bi, grouped, L, r, p);
            if (valid) load_particle();
        }
        float t[3] = {0.0f, 0.0f, 0.0f};
        uint32_t key = 0;
        if (valid) {
            frac_of(S, Xp, gxc, gyc, gzc, t);
            key = slot_key(S, code);
        }
        // ---- deformation-gradient update from the remapped velocities (MUSL)
        float Lg[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}; // dF/dt of the update
        if (use_r && valid) {
            uint32_t kprev = (code & TL_PREV_BIT) ? slot_key(S, D.code_prev[p]) : key;
            for (int k = 0; k < 8; k++) {
                float wx, wy, wz;
                corner_weights(t, k, wx, wy, wz);
                if (wx * wy * wz == 0.0f) continue;
                int bn = box_index(L.cxl + (k & 1), L.cyl + ((k >> 1) & 1), L.czl + ((k >> 2) & 1));
                int sl = find_slot(Tr, bn, kprev);
                if (sl < 0) {
                    atomicOr(D.status, TL_ST_LOOKUP);
                    continue;
                }
                float g0 = ((k & 1) ? S.inv_dx : -S.inv_dx) * wy * wz;
                float g1 = ((k & 2) ? S.inv_dx : -S.inv_dx) * wx * wz;
                float g2 = ((k & 4) ? S.inv_dx : -S.inv_dx) * wx * wy;
                for (int a = 0; a < 3; a++) {
                    float va = s_vt[sl * 3 + a];
                    Lg[3 * a + 0] += va * g0;
                    Lg[3 * a + 1] += va * g1;
                    Lg[3 * a + 2] += va * g2;
                }
            }
            bool fin = true;
            for (int a = 0; a < 9; a++) {
                H[a] += dt * Lg[a];
                D.H[a * N + p] = H[a];
                fin = fin && isfinite(H[a]);
            }
            if (!fin) atomicOr(D.status, TL_ST_NONFINITE);
            if (code & TL_PREV_BIT) {
                code &= ~TL_PREV_BIT;
                D.code[p] = code;
            }
        }
        // plasticity: F_p^{-1} = I + Gp; projection after each F update
        float Gp[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        if constexpr (MAT == 1) {
            if (S.ystress > 0.0f && valid) {
#pragma unroll
                for (int a = 0; a < 9; a++) Gp[a] = D.Gp[a * N + p];
                if (use_r) {
                    float K[9]; // F_e - I = H + Gp + H Gp
#pragma unroll
                    for (int i = 0; i < 3; i++)
#pragma unroll
                        for (int j = 0; j < 3; j++) {
                            float k = H[3 * i + j] + Gp[3 * i + j];
#pragma unroll
                            for (int m = 0; m < 3; m++) k += H[3 * i + m] * Gp[3 * m + j];
                            K[3 * i + j] = k;
                        }
                    const float Ey = S.e_uniform ? S.E0 : D.E[p];
                    if (vm_project(Ey, S.nu, S.ystress, K, Gp))
#pragma unroll
                        for (int a = 0; a < 9; a++) D.Gp[a * N + p] = Gp[a];
                }
            }
        }
        if constexpr (MAT == 1) {
            // viscosity uses the rate of the last F update: kept for the substeps
            // whose P2G has no pending update (the first, or after a state read)
            if (S.visc > 0.0f && valid) {
                if (use_r) {
#pragma unroll
                    for (int a = 0; a < 9; a++) D.Fdot[a * N + p] = Lg[a];
                } else {
#pragma unroll
                    for (int a = 0; a < 9; a++) Lg[a] = D.Fdot[a * N + p];
                }
            }
        }
        if (!A.do_p2g) continue;
        // ---- stress and external/contact impulses
        float m = 0.0f, V0 = 0.0f, E = 0.0f;
        float Pk[9];
        float Jc[3] = {0.0f, 0.0f, 0.0f};
        if (valid) {
            m = S.m_uniform ? S.m0 : D.m[p];
            V0 = S.v_uniform ? S.V0 : D.V0[p];
            E = S.e_uniform ? S.E0 : D.E[p];
            bool ok;
            if constexpr (MAT == 1) {
                if (S.ystress > 0.0f) {
                    // P = P_fcr(F_e) F_p^{-T}, F_e - I = H + Gp + H Gp, F_p^{-1} = I + Gp
                    float K[9], Pe[9];
#pragma unroll
                    for (int i = 0; i < 3; i++)
#pragma unroll
                        for (int j = 0; j < 3; j++) {
                            float k = H[3 * i + j] + Gp[3 * i + j];
#pragma unroll
                            for (int m = 0; m < 3; m++) k += H[3 * i + m] * Gp[3 * m + j];
                            K[3 * i + j] = k;
                        }
                    ok = fixed_corotated(E, S.nu, K, Pe);
#pragma unroll
                    for (int i = 0; i < 3; i++)
#pragma unroll
                        for (int j = 0; j < 3; j++) {
                            float a = Pe[3 * i + j];
#pragma unroll
                            for (int m = 0; m < 3; m++) a += Pe[3 * i + m] * Gp[3 * j + m];
                            Pk[3 * i + j] = a;
                        }
                } else {
                    ok = S.material == 1 ? fixed_corotated(E, S.nu, H, Pk) : neo_hookean(E, S.nu, H, Pk);
                }
            } else {
                ok = neo_hookean(E, S.nu, H, Pk);
            }
            if (ok && MAT == 1 && S.visc > 0.0f) add_viscous(S.visc, H, Lg, Pk);
            if (!ok) {
                atomicOr(D.status, TL_ST_NONFINITE);
                for (int a = 0; a < 9; a++) Pk[a] = 0.0f;
            }
        } else {
            for (int a = 0; a < 9; a++) Pk[a] = 0.0f;
        }
        float ext[3] = {0.0f, 0.0f, 0.0f};
        if (valid) {
            if (rig) { // floor and tool impulses of this substep (k_rigid)
                Jc[0] += D.Jrig[p];
                Jc[1] += D.Jrig[N + p];
                Jc[2] += D.Jrig[2 * N + p];
            }
            if (S.material_contact && (code & TL_CAND_BIT)) {
                Jc[0] += D.Jmat[p];
                Jc[1] += D.Jmat[N + p];
                Jc[2] += D.Jmat[2 * N + p];
            }
            ext[0] = Jc[0] + dt * m * S.gx;
            ext[1] = Jc[1] + dt * m * S.gy;
            ext[2] = Jc[2] + dt * m * S.gz;
        }
        // A = -dt V0 P;  dp_k = A grad N_k + w_k ext  (Eq. 2); a zero weight contributes
        // nothing (reading R7)
        const float sA = -dt * V0;
#pragma unroll
        for (int a = 0; a < 9; a++) Pk[a] *= sA;
        const float mm = valid ? m : 0.0f;
        // absolute corners (the CornerW order needs more registers here than the
        // selects it saves: the impulse generator also needs per-lane gradient signs)
        auto gen_mp = [&](int k, float* o) { // mass and momentum
            float wx, wy, wz;
            corner_weights(t, k, wx, wy, wz);
            float wm = wx * wy * wz * mm;
            o[0] = wm;
            o[1] = wm * vel[0];
            o[2] = wm * vel[1];
            o[3] = wm * vel[2];
        };
        auto gen_dp = [&](int k, float* o) { // internal, external and contact impulse
            float wx, wy, wz;
            corner_weights(t, k, wx, wy, wz);
            float w = wx * wy * wz;
            float g0 = ((k & 1) ? S.inv_dx : -S.inv_dx) * wy * wz;
            float g1 = ((k & 2) ? S.inv_dx : -S.inv_dx) * wx * wz;
            float g2 = ((k & 4) ? S.inv_dx : -S.inv_dx) * wx * wy;
            bool on = valid && w != 0.0f;
#pragma unroll
            for (int a = 0; a < 3; a++) {
                float f = Pk[3 * a] * g0 + Pk[3 * a + 1] * g1 + Pk[3 * a + 2] * g2 + w * ext[a];
                o[a] = on ? f : 0.0f;
            }
        };
        // impulses first: their butterfly then runs while fewer values are live;
        // stored as (m, m v, dp) like the other order
        accumulate_classes<3, 4, false, 4>(L, valid, key, gen_dp, gen_mp, T, s_acc, D.status);
    }
    if (!A.do_p2g) return;
    if (SPLIT && part == 0 && tid == 0) D.xp2g[bi] = split ? 1 : 0;
    write_partials<7>(S, part ? D.p2g_x : D.p2g, bi, T, total_c, s_acc);
}

// --------------------------------------------------------------------------- K_B
// Grid update and G2P kernel (one brick per workgroup): finalize the box from the
// P2G partials (sum over contributing bricks, coupling Eq. 8, velocities Eq. 9),
// PIC/FLIP G2P of v and x (Eq. 17), then the MUSL re-scatter of m_p v_p^{n+1} into
// this brick's partials.  Also records the brick's current AABB and speed bound.
template <bool SPLIT>
DEV void g2p_body(const SceneK& S, const SceneD& D, int bi, int cur, int part)
{
    __shared__ BoxTab T;
    __shared__ float s_sum[TL_BOX_SLOTS * 7];
    __shared__ float s_grid[TL_BOX_SLOTS * 6];
    __shared__ float s_acc[TL_BOX_SLOTS * 4];
    __shared__ int s_total;
    __shared__ int s_nb[27];
    __shared__ int s_rounds;
    __shared__ float s_bb[8][8];

    const int nround = SPLIT ? D.bround[bi] : 0; // rounds of a brick with a mixed cell, else 0
    if (SPLIT && part == 1 && nround <= 1) return; // (split bricks as in the P2G)
    const int brick = D.active[bi];
    if (bi == 0 && part == 0 && threadIdx.x == 0) {
        // end of the substep for this scene: next history stamp, F update pending
        // (no other kernel of the substep reads these after this point); whether this
        // G2P splits its mixed bricks (read by the next P2G and box tests)
        D.ctr[0] += 1;
        D.ctr[1] = 1;
        D.ctr[2] += 1;
        if (SPLIT) D.xg[0] = (S.xcap > 0 && D.ctr[3] > 0 && D.ctr[3] <= S.xcap) ? 1 : 0;
    }
    const bool grouped = D.bmixed[brick] != 0; // a cell holds two codes: same-code groups
    // this substep's P2G split its mixed bricks (a scene without split workgroups never)
    const bool xsplit = SPLIT && S.xcap > 0 && D.ctr[3] > 0 && D.ctr[3] <= S.xcap;
    const bool split = grouped && nround > 1 && xsplit;
    const int r0 = part;
    const int bx = brick % S.cbx, by = (brick / S.cbx) % S.cby, bz = brick / (S.cbx * S.cby);
    const int tid = threadIdx.x;
    const long long N = S.N;
    const float dt = S.dt, beta = S.beta;
    // displacement anchor of this workgroup's particles (pair-search skip), kept for
    // bricks with contact candidates (only candidates can be partners): the centre of
    // the brick's box after the last G2P minus the centre of its particles' reference
    // box.  A split brick's second workgroup reads the first one's record, which that
    // one may rewrite in this launch; either value is a valid anchor, since the spread
    // is measured against the anchor taken.
    const bool track = S.pair_skip && D.bcand[bi] > 0;
    float ap[3] = {0.0f, 0.0f, 0.0f};
    if (track) g2p_anchor(D, D.aabb + (long long)brick * 8, brick, ap);

    // ---- phase 1: cell index, box counts, round-0 particle loads
    Lane L = lane_of(D, brick);
    box_counts(S, D.cnt[cur], bx, by, bz, T);
    load_neighbours(S, D, bx, by, bz, s_nb);
    if (tid == 0) s_rounds = 0;
    const int gxc = bx * TL_B + L.cxl, gyc = by * TL_B + L.cyl, gzc = bz * TL_B + L.czl;
    long long p = L.beg;
    bool valid = lane_particle(D, bi, grouped, L, r0, p);
    float Xp[3] = {0.0f, 0.0f, 0.0f}, v[3] = {0.0f, 0.0f, 0.0f}, u[3] = {0.0f, 0.0f, 0.0f};
    uint32_t code = 0;
    auto load_particle = [&]() {
        for (int a = 0; a < 3; a++) {
            Xp[a] = D.X[a * N + p];
            v[a] = D.v[a * N + p];
            u[a] = D.u[a * N + p];
        }
        code = D.code[p];
    };
    if (valid) load_particle();
    lds_barrier();
    if (grouped) {
        if (tid == 0) s_rounds = D.bround[bi];
    } else if (L.j == 0) {
        atomicMax(&s_rounds, (L.count + 7) >> 3);
    }
    box_scan(T, &s_total, 0);
    lds_barrier();
    const int total = s_total;
    if (total > TL_BOX_SLOTS) {
        if (tid == 0) atomicOr(D.status, TL_ST_BOX);
        return;
    }
    // ---- phase 3: per box node: codes, P2G sums, coupling (Eq. 8), v^n and dv (Eq. 9)
    if ((tid >> 2) < TL_BOXN) {
        const int bn = tid >> 2, u = tid & 3;
        uint32_t pre[2];
        if (u == 0) codes_pre(S, D.scode[cur], T, bn, pre);
        const int c = T.cnt[bn], b0 = T.base[bn];
        if (c > 0) gather_node4<7>(S, s_nb, D.p2g, D.p2g_x, xsplit ? D.xp2g : nullptr, T, bn, u, s_sum);
        if (u == 0) codes_put(S, D.scode[cur], T, bn, pre);
        if (u == 0 && c > 0) {
            float* gvn = s_grid;
            float* gdv = s_grid + TL_BOX_SLOTS * 3;
            couple_node<7>(T, b0, c, s_sum, 1, gvn);
            couple_node<7>(T, b0, c, s_sum, 4, gdv);
            for (int a = 0; a < c; a++) {
                float m = s_sum[(b0 + a) * 7];
                float im = m > 0.0f ? 1.0f / m : 0.0f;
                for (int jj = 0; jj < 3; jj++) {
                    gvn[(b0 + a) * 3 + jj] *= im;
                    gdv[(b0 + a) * 3 + jj] *= im;
                }
            }
        }
    }
    for (int q = tid; q < total * 4; q += TL_WG) s_acc[q] = 0.0f;
    lds_barrier();
    const int rounds = (split && part == 0) ? 1 : s_rounds;
    // box of x^{n+1}, speed bound, and the largest |u^{n+1} - a| about the anchor a
    // (for the pair-search skip)
    float bb[8] = {1e30f, 1e30f, 1e30f, -1e30f, -1e30f, -1e30f, 0.0f, 0.0f};
    const float* gv = s_grid;
    const float* gdv = s_grid + TL_BOX_SLOTS * 3;
    for (int r = r0; r < rounds; r++) {
        if (r > r0) {
            valid = lane_particle(D, bi, grouped, L, r, p);
            if (valid) load_particle();
        }
        float t[3] = {0.0f, 0.0f, 0.0f};
        uint32_t key = 0;
        float m = 0.0f, vn1[3] = {0.0f, 0.0f, 0.0f};
        if (valid) {
            frac_of(S, Xp, gxc, gyc, gzc, t);
            key = slot_key(S, code);
            float av[3] = {0.0f, 0.0f, 0.0f}, ax[3] = {0.0f, 0.0f, 0.0f};
            for (int k = 0; k < 8; k++) {
                float wx, wy, wz;
                corner_weights(t, k, wx, wy, wz);
                float w = wx * wy * wz;
                if (w == 0.0f) continue;
                int bn = box_index(L.cxl + (k & 1), L.cyl + ((k >> 1) & 1), L.czl + ((k >> 2) & 1));
                int sl = find_slot(T, bn, key);
                if (sl < 0) {
                    atomicOr(D.status, TL_ST_LOOKUP);
                    continue;
                }
                for (int a = 0; a < 3; a++) {
                    float vn = gv[sl * 3 + a], dv = gdv[sl * 3 + a];
                    av[a] += w * ((1.0f - beta) * vn + dv);
                    ax[a] += w * (vn + dv);
                }
            }
            for (int a = 0; a < 3; a++) {
                vn1[a] = beta * v[a] + av[a];
                float un = u[a] + dt * ax[a];
                D.v[a * N + p] = vn1[a];
                D.u[a * N + p] = un;
                float xa = Xp[a] + un;
                bb[a] = fminf(bb[a], xa);
                bb[3 + a] = fmaxf(bb[3 + a], xa);
                bb[7] = fmaxf(bb[7], fabsf(un - ap[a]));
            }
            bb[6] = fmaxf(bb[6], sqrtf(vn1[0] * vn1[0] + vn1[1] * vn1[1] + vn1[2] * vn1[2]));
            m = S.m_uniform ? S.m0 : D.m[p];
        }
        const float mm = valid ? m : 0.0f;
        const CornerW cw = corner_table(t, L.j);
        auto gen = [&](int r, float* o) {
            const float wx = cw.wx[r & 1], wy = cw.wy[(r >> 1) & 1], wz = cw.wz[r >> 2];
            float w = wx * wy * wz * mm;
            o[0] = w;
            o[1] = w * vn1[0];
            o[2] = w * vn1[1];
            o[3] = w * vn1[2];
        };
        accumulate_classes<4, 0, true>(L, valid, key, gen, gen, T, s_acc, D.status);
    }
    if (SPLIT && part == 0 && tid == 0) D.xrs[bi] = split ? 1 : 0;
    write_partials<4>(S, part ? D.rs_x : D.rs, bi, T, total, s_acc);
    // brick AABB of x^{n+1} and speed bound (used to skip distant contact work); a
    // split brick's second workgroup keeps the box of its particles apart
    // (brick_aabb joins the two)
#pragma unroll
    for (int q = 0; q < 8; q++) {
        if (q == 7 && !track) break;
        float val = bb[q];
        auto mm = [&](float other) { val = (q < 3) ? fminf(val, other) : fmaxf(val, other); };
        mm(lane_xor<1>(val));
        mm(lane_xor<2>(val));
        mm(lane_xor<4>(val));
        for (int o = 8; o <= 32; o <<= 1) mm(__shfl_xor(val, o, 64));
        if (L.lane == 0) s_bb[L.w][q] = val;
    }
    lds_barrier();
    if (tid < 7) {
        float val = s_bb[0][tid];
        for (int wv = 1; wv < 8; wv++) val = (tid < 3) ? fminf(val, s_bb[wv][tid]) : fmaxf(val, s_bb[wv][tid]);
        (part ? D.aabb_x : D.aabb)[(long long)brick * 8 + tid] = val;
        // the next binning's bin edge needs the largest speed bound; the maximum
        // of non-negative floats is taken on their bit patterns (order-independent)
        if (tid == 6 && S.material_contact && val > 0.0f)
            atomicMax(D.hmax + (bi & (TL_HSLOTS - 1)) * TL_HSTRIDE, __float_as_int(val));
    } else if (tid == 7 && track) {
        float dv = s_bb[0][7];
        for (int wv = 1; wv < 8; wv++) dv = fmaxf(dv, s_bb[wv][7]);
        put_anchor(D, bi, brick, part, ap, dv);
    }
}

// ------------------------------------------------------------- mixed-code bricks
// Per cell of a brick whose codes changed (or of every brick, when forced): the
// one slot key of its particles (or empty / mixed).  A brick with a mixed cell
// gets a group table: each of its cells lists its particles by ascending key
// (input order within a key) in gperm over the cell's range, cut into groups of at
// most 8 same-key particles; P2G and G2P then take one group per cell and round.
DEV void cell_summaries(const SceneK& S, const SceneD& D, int bi, int brick)
{
    __shared__ int s_rounds;
    __shared__ uint32_t s_bor;
    if (threadIdx.x == 0) {
        s_rounds = 1;
        s_bor = 0u;
    }
    __syncthreads();
    bool mixed = false;
    for (int c = threadIdx.x; c < TL_CELLS; c += blockDim.x) {
        const long long cs = (long long)brick * TL_CELLS + c;
        const int b0 = D.cell_start[cs], b1 = D.cell_start[cs + 1];
        if (b1 <= b0) {
            D.ccode[cs] = TL_CC_EMPTY;
            if (S.material_contact) D.cmask[cs] = 0;
            continue;
        }
        const uint32_t k0 = slot_key(S, D.code[b0]);
        uint32_t orm = k0; // OR of the codes of the cell (material contact candidates)
        uint32_t ks[TL_CKEYS] = {k0, 0u, 0u, 0u};
        int nk = 1;
        bool many = false;
#pragma unroll 4
        for (int p = b0 + 1; p < b1; p++) {
            const uint32_t k = slot_key(S, D.code[p]);
            orm |= k;
            // distinct keys in ascending order (insertion; at most TL_CKEYS kept)
            bool seen = false;
#pragma unroll
            for (int q = 0; q < TL_CKEYS; q++) seen |= q < nk && ks[q] == k;
            if (seen) continue;
            if (nk == TL_CKEYS) {
                many = true;
                continue;
            }
#pragma unroll
            for (int q = TL_CKEYS - 1; q > 0; q--)
                if (q <= nk && ks[q - 1] > k) {
                    ks[q] = ks[q - 1];
                    ks[q - 1] = k;
                } else if (q == nk) {
                    ks[q] = k;
                }
            nk++;
        }
        const bool cm = nk > 1 || many;
        D.ccode[cs] = !cm ? k0 : (many ? TL_CC_MIXED : (TL_CC_FEW | (uint32_t)nk));
        if (cm && !many)
            for (int q = 0; q < nk; q++) D.ckeys[cs * TL_CKEYS + q] = ks[q];
        if (S.material_contact) D.cmask[cs] = orm;
        if (S.pair_skip && orm) atomicOr(&s_bor, orm);
        mixed |= cm;
    }
    const int m = __syncthreads_or(mixed);
    if (threadIdx.x == 0) {
        if (S.pair_skip) D.bor[brick] = s_bor; // (the barrier above ordered the LDS ORs)
        D.bmixed[brick] = m;
        if (!m) {
            D.bround[bi] = 0; // no split workgroup for this brick
        } else if (S.xcap > 0 && !D.xin[bi]) { // (codes only gain digits: once mixed, always mixed)
            D.xin[bi] = 1;
            D.xlist[atomicAdd(D.ctr + 3, 1)] = bi;
        }
    }
    if (!m) return;
    if (threadIdx.x < TL_CELLS) {
        const int c = threadIdx.x; // cell slot w * 8 + i
        const long long cs = (long long)brick * TL_CELLS + c;
        const int b0 = D.cell_start[cs], b1 = D.cell_start[cs + 1];
        int* meta = D.gmeta + ((long long)bi * TL_CELLS + c) * TL_GMAX;
        const int n = b1 - b0;
        // the keys of the cell's first TL_KC particles, loaded once (registers: every
        // index below is a compile-time constant); the rest are read when needed
        constexpr int TL_KC = 8;
        uint32_t kc[TL_KC];
#pragma unroll
        for (int q = 0; q < TL_KC; q++) kc[q] = q < n ? slot_key(S, D.code[b0 + q]) : 0u;
        int ng = 0, pos = 0, gstart = 0;
        uint32_t last = 0;
        bool first = true;
        auto place = [&](int p) {
            D.gperm[b0 + pos] = p;
            pos++;
            if (pos - gstart == 8) {
                if (ng < TL_GMAX) meta[ng] = (gstart << 4) | 8;
                ng++;
                gstart = pos;
            }
        };
        while (pos < n) {
            uint32_t kmin = 0xFFFFFFFFu; // smallest key above the last one
#pragma unroll
            for (int q = 0; q < TL_KC; q++)
                if (q < n && (first || kc[q] > last) && kc[q] < kmin) kmin = kc[q];
            for (int q = TL_KC; q < n; q++) {
                const uint32_t k = slot_key(S, D.code[b0 + q]);
                if ((first || k > last) && k < kmin) kmin = k;
            }
            gstart = pos;
#pragma unroll
            for (int q = 0; q < TL_KC; q++)
                if (q < n && kc[q] == kmin) place(b0 + q);
            for (int q = TL_KC; q < n; q++)
                if (slot_key(S, D.code[b0 + q]) == kmin) place(b0 + q);
            if (pos > gstart) {
                if (ng < TL_GMAX) meta[ng] = (gstart << 4) | (pos - gstart);
                ng++;
            }
            last = kmin;
            first = false;
        }
        for (int g = ng; g < TL_GMAX; g++) meta[g] = 0;
        if (ng > TL_GMAX) atomicOr(D.status, TL_ST_BOX);
        atomicMax(&s_rounds, ng < TL_GMAX ? ng : TL_GMAX);
    }
    __syncthreads();
    if (threadIdx.x == 0) D.bround[bi] = s_rounds;
}

DEV void mixed_body(const SceneK& S, const SceneD& D, int bi, int force)
{
    const int brick = D.active[bi];
    if (!force && D.bdirty[brick] != D.ctr[0]) return;
    cell_summaries(S, D, bi, brick);
}

// ------------------------------------------------------------------------ labels
// Side-label pass (Eqs. 3, 4, 6) with the predicates of tlmpm_band.h (FP64, a
// fixed evaluation order, no contraction: the order of the CPU reference), on
// x = X + u and v.  One brick per workgroup; a brick whose box cannot meet any band
// exits at once.
// Blade of tool b at this substep (TL_TOOL_ADVANCE translates the edge).
DEV DevBlade blade_at(const DevTool& T, double jdt)
{
    DevBlade B = T.b;
    if (T.flags & TL_TOOL_ADVANCE)
        for (int a = 0; a < 3; a++) B.xe[a] = T.b.xe[a] + jdt * T.b.ve[a];
    return B;
}

// Blades whose band can reach active brick bi (= brick) this substep: bit b for
// tools[b] (label tools only; brick_near_band, conservative).
DEV int label_mask(const SceneK& S, const SceneD& D, int bi, int brick, int n_tools, double jdt)
{
    float bb[7];
    brick_aabb(S, D, bi, brick, bb);
    int m = 0;
    for (int b = 0; b < n_tools; b++) {
        if (!(D.tools[b].flags & TL_TOOL_LABELS)) continue;
        if (brick_near_band(bb, blade_at(D.tools[b], jdt), S.dt_d)) m |= 1 << b;
    }
    return m;
}

// Label pass of one brick within reach of the blades of mask m (whole block).
DEV void labels_brick(const SceneK& S, const SceneD& D, int bi, int brick, int m, double jdt)
{
    const bool mark_prev = D.ctr[1] != 0; // keep the codes the pending F update needs
    __shared__ DevBlade s_bl[TL_MAX_TOOLS];
    __shared__ int s_nb;
    if (threadIdx.x == 0) {
        int nb = 0;
        for (int b = 0; b < TL_MAX_TOOLS; b++)
            if ((m >> b) & 1) s_bl[nb++] = blade_at(D.tools[b], jdt);
        s_nb = nb;
    }
    __syncthreads();
    const long long N = S.N;
    const int beg = D.cell_start[(long long)brick * TL_CELLS], end = D.cell_start[(long long)(brick + 1) * TL_CELLS];
    bool any = false;
    for (int p = beg + threadIdx.x; p < end; p += blockDim.x) {
        uint32_t code = D.code[p];
        uint32_t nc = code;
        double x[3] = {(double)D.X[p] + (double)D.u[p], (double)D.X[N + p] + (double)D.u[N + p],
                       (double)D.X[2 * N + p] + (double)D.u[2 * N + p]};
        double v[3] = {(double)D.v[p], (double)D.v[N + p], (double)D.v[2 * N + p]};
        for (int b = 0; b < s_nb; b++) {
            const DevBlade& B = s_bl[b];
            uint32_t bit1 = 1u << B.cut, bit2 = 1u << (15 + B.cut);
            if (nc & (bit1 | bit2)) continue; // persistence: an assigned digit never changes
            int dg = label_digit(x, v, B, S.dt_d);
            if (dg == 1) nc |= bit1;
            if (dg == 2) nc |= bit2;
        }
        if (nc != code) {
            if (mark_prev && !(code & TL_PREV_BIT)) {
                D.code_prev[p] = code & TL_CODE_MASK;
                nc |= TL_PREV_BIT;
            }
            D.code[p] = nc;
            any = true;
        }
    }
    if (__syncthreads_or(any)) {
        // label-change flags carry the substep stamp: no clearing pass needed
        if (threadIdx.x == 0) D.bdirty[brick] = D.ctr[0];
        __syncthreads(); // the new codes of the brick, visible to the whole block
        cell_summaries(S, D, bi, brick);
    }
}

DEV void labels_body(const SceneK& S, const SceneD& D, int bi)
{
    const double jdt = (double)D.ctr[2] * S.dt_d; // substep of the call (TL_TOOL_ADVANCE poses)
    __shared__ int s_m;
    const int brick = D.active[bi];
    if (threadIdx.x == 0) s_m = label_mask(S, D, bi, brick, D.tinfo[0], jdt);
    __syncthreads();
    const int m = s_m;
    if (!m) return;
    labels_brick(S, D, bi, brick, m, jdt);
}

// Label pass of one scene with TL_LBRICKS bricks per workgroup: the first lanes test
// the bands of bricks w, w + G, w + 2G, ... (G workgroups: the bricks of a blade's
// band, neighbours in the active order, fall to different workgroups), then the
// workgroup labels the bricks within reach one after another.  Far fewer workgroups
// than bricks, most of which only test.
#define TL_LBRICKS 16
__global__ __launch_bounds__(256) void k_labels_multi(SceneK S, SceneD D)
{
    __shared__ int s_m[TL_LBRICKS];
    const double jdt = (double)D.ctr[2] * S.dt_d;
    const int G = gridDim.x;
    if (threadIdx.x < TL_LBRICKS) {
        const int bi = blockIdx.x + threadIdx.x * G;
        s_m[threadIdx.x] = bi < D.n_active ? label_mask(S, D, bi, D.active[bi], D.tinfo[0], jdt) : 0;
    }
    __syncthreads();
    for (int k = 0; k < TL_LBRICKS; k++) {
        const int m = s_m[k];
        if (!m) continue;
        const int bi = blockIdx.x + k * G;
        labels_brick(S, D, bi, D.active[bi], m, jdt);
        __syncthreads(); // the brick's LDS words are reused by the next one
    }
}

// The same over the n (scene, brick) work items of a batch.
__global__ __launch_bounds__(256) void k_labels_multi_b(const SceneK* __restrict__ Ks, const SceneD* __restrict__ Ds,
                                                        const int2* __restrict__ it, int n)
{
    __shared__ int s_m[TL_LBRICKS];
    const int G = gridDim.x;
    if (threadIdx.x < TL_LBRICKS) {
        const int i = blockIdx.x + threadIdx.x * G;
        int m = 0;
        if (i < n) {
            const int2 t = it[i];
            const SceneK& S = Ks[t.x];
            const SceneD& D = Ds[t.x];
            m = label_mask(S, D, t.y, D.active[t.y], D.tinfo[0], (double)D.ctr[2] * S.dt_d);
        }
        s_m[threadIdx.x] = m;
    }
    __syncthreads();
    for (int k = 0; k < TL_LBRICKS; k++) {
        const int m = s_m[k];
        if (!m) continue;
        const int2 t = it[blockIdx.x + k * G];
        const SceneK& S = Ks[t.x];
        const SceneD& D = Ds[t.x];
        labels_brick(S, D, t.y, D.active[t.y], m, (double)D.ctr[2] * S.dt_d);
        __syncthreads();
    }
}

// --------------------------------------------------------------- small kernels
// D := 0 for a new cut (Sec. III-A), over particle block bi
DEV void resetD_body(const SceneK& S, const SceneD& D, int bi)
{
    if (!D.tinfo[2]) return;
    long long i = (long long)bi * blockDim.x + threadIdx.x;
    if (i < S.N) D.D[i] = 0.0f;
}

// start of a call: substep index 0 and (with tool contact) a cleared interval
// wrench accumulator
DEV void call_start_body(const SceneK& S, const SceneD& D, int bi)
{
    if (threadIdx.x == 0) D.ctr[2] = 0;
    if (D.tinfo[1] && threadIdx.x < TL_MAX_TOOLS * 6) D.wacc[threadIdx.x] = 0.0;
}

// Workspace of the batches that allocate no device memory (tlmpm_batch_create_static):
// one array per GPU, held by at most one such batch at a time, for the life of the
// process.  Its size bounds their footprint (TL_STATIC_SCRATCH_BYTES).
static __device__ __align__(256) unsigned char scratch[TL_STATIC_SCRATCH_BYTES];

__global__ void k_fill_f32(float* p, long long n, float v)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_i32(int* p, long long n, int v)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// brick AABB from the current state (scene creation, after a state write); with the
// pair-search skip also the centre of the box of the reference positions and the
// displacement anchor (exact spread: a second pass over the particles)
DEV void aabb_body(const SceneK& S, const SceneD& D, int bi)
{
    __shared__ float s_bb[4][13];
    __shared__ float s_a[3];
    const int brick = D.active[bi];
    const long long N = S.N;
    const int beg = D.cell_start[(long long)brick * TL_CELLS], end = D.cell_start[(long long)(brick + 1) * TL_CELLS];
    // current box (0-5), speed (6), reference box (7-12)
    float bb[13] = {1e30f, 1e30f, 1e30f, -1e30f, -1e30f, -1e30f, 0.0f, 1e30f, 1e30f, 1e30f, -1e30f, -1e30f, -1e30f};
    for (int p = beg + threadIdx.x; p < end; p += blockDim.x) {
        float sp = 0.0f;
        for (int a = 0; a < 3; a++) {
            const float X = D.X[a * N + p];
            float xa = X + D.u[a * N + p];
            bb[a] = fminf(bb[a], xa);
            bb[3 + a] = fmaxf(bb[3 + a], xa);
            bb[7 + a] = fminf(bb[7 + a], X);
            bb[10 + a] = fmaxf(bb[10 + a], X);
            sp += D.v[a * N + p] * D.v[a * N + p];
        }
        bb[6] = fmaxf(bb[6], sqrtf(sp));
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    auto is_min = [](int q) { return q < 3 || (q >= 7 && q < 10); };
    for (int q = 0; q < 13; q++) {
        float val = bb[q];
        for (int o = 32; o >= 1; o >>= 1) {
            float other = __shfl_xor(val, o, 64);
            val = is_min(q) ? fminf(val, other) : fmaxf(val, other);
        }
        if (lane == 0) s_bb[w][q] = val;
    }
    __syncthreads();
    if (threadIdx.x < 13) {
        int q = threadIdx.x;
        float val = s_bb[0][q];
        for (int wv = 1; wv < 4; wv++) val = is_min(q) ? fminf(val, s_bb[wv][q]) : fmaxf(val, s_bb[wv][q]);
        if (q < 7) D.aabb[(long long)brick * 8 + q] = val;
        if (q == 6 && S.material_contact && val > 0.0f)
            atomicMax(D.hmax + (bi & (TL_HSLOTS - 1)) * TL_HSTRIDE, __float_as_int(val));
        s_bb[0][q] = val;
    }
    if (!S.pair_skip) return;
    __syncthreads();
    if (threadIdx.x < 3) { // (the anchor g2p_anchor would form from this box)
        const int a = threadIdx.x;
        const float rc = 0.5f * (s_bb[0][7 + a] + s_bb[0][10 + a]);
        D.uref[(long long)brick * 4 + a] = rc;
        s_a[a] = 0.5f * (s_bb[0][a] + s_bb[0][3 + a]) - rc;
    }
    __syncthreads();
    // spread about the anchor: exact, from a second pass over the particles
    float dv = 0.0f;
    for (int p = beg + threadIdx.x; p < end; p += blockDim.x)
        for (int a = 0; a < 3; a++) dv = fmaxf(dv, fabsf(D.u[a * N + p] - s_a[a]));
    for (int o = 32; o >= 1; o >>= 1) dv = fmaxf(dv, __shfl_xor(dv, o, 64));
    __syncthreads();
    if (lane == 0) s_bb[w][7] = dv;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int wv = 1; wv < 4; wv++) dv = fmaxf(dv, s_bb[wv][7]);
        const float a[3] = {s_a[0], s_a[1], s_a[2]};
        put_anchor(D, bi, brick, 0, a, dv);
    }
}

// Once per call: sum of the per-brick wrench partials accumulated over the call's
// substeps, in fixed order (one workgroup per force or torque component: four
// running sums per thread, a tree over the workgroup), added to the interval
// accumulator; the partials are cleared for the next call.
DEV void wrench_body(const SceneK& S, const SceneD& D, int bi)
{
    __shared__ double s[256];
    const int q = bi;
    if (!D.tinfo[1] || q >= D.tinfo[0] * 6) return;
    double* w = D.wpart + (long long)q * D.n_active;
    const int n = D.n_active, T = blockDim.x;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int b = threadIdx.x;
    for (; b + 3 * T < n; b += 4 * T) {
        a0 += w[b];
        a1 += w[b + T];
        a2 += w[b + 2 * T];
        a3 += w[b + 3 * T];
        w[b] = 0.0;
        w[b + T] = 0.0;
        w[b + 2 * T] = 0.0;
        w[b + 3 * T] = 0.0;
    }
    for (; b < n; b += T) {
        a0 += w[b];
        w[b] = 0.0;
    }
    s[threadIdx.x] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) D.wacc[q] += s[0];
}

// ------------------------------------------------------------------- kernels
// Every body runs either for one scene (parameters by value, block = item) or for
// a batch (block -> (scene, item) from a list).
#define TL_WRAP(NAME, BOUNDS, PARAMS, ARGS)                                                                   \
    __global__ __launch_bounds__(BOUNDS) void k_##NAME(SceneK S, SceneD D PARAMS)                           \
    {                                                                                                       \
        NAME##_body(S, D, blockIdx.x ARGS);                                                                 \
    }                                                                                                       \
    __global__ __launch_bounds__(BOUNDS) void k_##NAME##_b(const SceneK* __restrict__ Ks,                    \
                                                           const SceneD* __restrict__ Ds,                    \
                                                           const int2* __restrict__ it PARAMS)               \
    {                                                                                                       \
        const int2 t = it[blockIdx.x];                                                                      \
        NAME##_body(Ks[t.x], Ds[t.x], t.y ARGS);                                                            \
    }

#define TL_COMMA ,
TL_WRAP(rigid, 256, , )
TL_WRAP(slots, 256, TL_COMMA int dst TL_COMMA int src TL_COMMA int force, TL_COMMA dst TL_COMMA src TL_COMMA force)
TL_WRAP(mixed, 256, TL_COMMA int force, TL_COMMA force)
TL_WRAP(aabb, 256, , )
TL_WRAP(wrench, 256, , )
TL_WRAP(resetD, 256, , )
TL_WRAP(call_start, 64, , )

// The label pass and rigid contact in one launch: blocks below nl take the label
// pass of a brick, the others its rigid contact.  Rigid contact reads only the last
// substep's motion, the tools and the cutting progress, none of which the label pass
// writes, and the label pass reads nothing rigid contact writes.
__global__ __launch_bounds__(256) void k_labels_rigid(SceneK S, SceneD D, int nl)
{
    if ((int)blockIdx.x < nl)
        labels_body(S, D, blockIdx.x);
    else
        rigid_body(S, D, blockIdx.x - nl);
}
__global__ __launch_bounds__(256) void k_labels_rigid_b(const SceneK* __restrict__ Ks, const SceneD* __restrict__ Ds,
                                                        const int2* __restrict__ it, int nl)
{
    const bool lb = (int)blockIdx.x < nl;
    const int2 t = it[lb ? blockIdx.x : blockIdx.x - nl];
    if (lb)
        labels_body(Ks[t.x], Ds[t.x], t.y);
    else
        rigid_body(Ks[t.x], Ds[t.x], t.y);
}

// at most 80 VGPRs: three 512-thread workgroups per CU
// Neo-Hookean: at most 80 VGPRs (three workgroups per CU); the general path (polar
// decomposition) at most 128 (two)
// P2G and G2P launch, ahead of the one workgroup per brick, S.xcap workgroups for the
// later rounds of the bricks in xlist (dispatched first so that these long ones start
// early).  Bricks are split only while all mixed bricks of the scene have such a
// workgroup (at most S.xcap of them); otherwise every brick keeps all its rounds, so
// the results do not depend on the order of xlist.  Block b -> (active index, part);
// -1: nothing to do.
DEV int brick_of_block(const SceneK& S, const SceneD& D, int b, int j, int& part)
{
    if (j < 0) {
        part = 0;
        return b;
    }
    part = 1;
    const int count = D.ctr[3];
    return (j < count && count <= S.xcap) ? D.xlist[j] : -1;
}

// SPLIT false: one workgroup per brick, every brick keeps all its rounds (scenes with
// S.xcap = 0, and batches of such scenes); true: the xcap extra workgroups first.
template <int MAT, bool SPLIT>
__global__ __launch_bounds__(TL_WG) __attribute__((amdgpu_waves_per_eu(MAT == 0 ? 6 : 4))) void k_p2g(SceneK S,
                                                                                                     SceneD D,
                                                                                                     KA_Args A)
{
    const int b = blockIdx.x;
    if constexpr (!SPLIT) {
        p2g_body<MAT, false>(S, D, b, A, 0);
    } else {
        int part;
        const int bi = brick_of_block(S, D, b - S.xcap, b < S.xcap ? b : -1, part);
        if (bi >= 0) p2g_body<MAT, true>(S, D, bi, A, part);
    }
}
template <int MAT, bool SPLIT>
__global__ __launch_bounds__(TL_WG) __attribute__((amdgpu_waves_per_eu(MAT == 0 ? 6 : 4))) void k_p2g_b(
    const SceneK* __restrict__ Ks, const SceneD* __restrict__ Ds, const int2* __restrict__ it,
    const int2* __restrict__ xit, int nx, KA_Args A)
{
    const int b = blockIdx.x;
    if constexpr (!SPLIT) {
        const int2 t = it[xcd_order(b, gridDim.x)];
        p2g_body<MAT, false>(Ks[t.x], Ds[t.x], t.y, A, 0);
    } else {
        const int2 t = b < nx ? xit[b] : it[xcd_order(b - nx, gridDim.x - nx)];
        int part;
        const int bi = brick_of_block(Ks[t.x], Ds[t.x], t.y, b < nx ? t.y : -1, part);
        if (bi >= 0) p2g_body<MAT, true>(Ks[t.x], Ds[t.x], bi, A, part);
    }
}
template <bool SPLIT>
__global__ __launch_bounds__(TL_WG) void k_g2p(SceneK S, SceneD D, int cur)
{
    const int b = blockIdx.x;
    if constexpr (!SPLIT) {
        g2p_body<false>(S, D, b, cur, 0);
    } else {
        int part;
        const int bi = brick_of_block(S, D, b - S.xcap, b < S.xcap ? b : -1, part);
        if (bi >= 0) g2p_body<true>(S, D, bi, cur, part);
    }
}
template <bool SPLIT>
__global__ __launch_bounds__(TL_WG) void k_g2p_b(const SceneK* __restrict__ Ks, const SceneD* __restrict__ Ds,
                                                 const int2* __restrict__ it, const int2* __restrict__ xit, int nx,
                                                 int cur)
{
    const int b = blockIdx.x;
    if constexpr (!SPLIT) {
        const int2 t = it[xcd_order(b, gridDim.x)];
        g2p_body<false>(Ks[t.x], Ds[t.x], t.y, cur, 0);
    } else {
        const int2 t = b < nx ? xit[b] : it[xcd_order(b - nx, gridDim.x - nx)];
        int part;
        const int bi = brick_of_block(Ks[t.x], Ds[t.x], t.y, b < nx ? t.y : -1, part);
        if (bi >= 0) g2p_body<true>(Ks[t.x], Ds[t.x], bi, cur, part);
    }
}

// ------------------------------------------------------------------- launchers
template <class KP, class KB, class... Args>
static hipError_t tl_run(const TlLaunch& L, int kind, int plain_blocks, int threads, KP kp, KB kb, Args... args)
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

// one workgroup per brick, plus (split kernels) the workgroups of the split bricks'
// later rounds
template <class KP, class KB, class KPX, class KBX, class... Args>
static hipError_t tl_run_split(const TlLaunch& L, KP kp, KB kb, KPX kpx, KBX kbx, Args... args)
{
    if (L.S) {
        if (L.D->n_active <= 0) return hipSuccess;
        if (L.S->xcap > 0)
            hipLaunchKernelGGL(kpx, dim3(L.S->xcap + L.D->n_active), dim3(TL_WG), 0, L.st, *L.S, *L.D, args...);
        else
            hipLaunchKernelGGL(kp, dim3(L.D->n_active), dim3(TL_WG), 0, L.st, *L.S, *L.D, args...);
    } else {
        if (L.n_items[IT_BRICK] <= 0) return hipSuccess;
        const int nx = L.n_items[IT_XBRICK];
        if (nx > 0)
            hipLaunchKernelGGL(kbx, dim3(nx + L.n_items[IT_BRICK]), dim3(TL_WG), 0, L.st, L.Ks, L.Ds,
                               L.items[IT_BRICK], L.items[IT_XBRICK], nx, args...);
        else
            hipLaunchKernelGGL(kb, dim3(L.n_items[IT_BRICK]), dim3(TL_WG), 0, L.st, L.Ks, L.Ds, L.items[IT_BRICK],
                               L.items[IT_XBRICK], 0, args...);
    }
    return hipGetLastError();
}

static int blocks_of(long long n, int per) { return (int)((n + per - 1) / per); }
static int plain_bricks(const TlLaunch& L) { return L.S ? L.D->n_active : 0; }
static int plain_nodes(const TlLaunch& L) { return L.S ? blocks_of(L.S->NN, 256) : 0; }
static int plain_parts(const TlLaunch& L) { return L.S ? blocks_of(L.S->N, 256) : 0; }
static int plain_bflags(const TlLaunch& L)
{
    return L.S ? blocks_of((long long)L.S->cbx * L.S->cby * L.S->cbz, 256) : 0;
}

extern "C" {
hipError_t tl_launch_rigid(const TlLaunch* L)
{
    return tl_run(*L, IT_BRICK, plain_bricks(*L), 256, k_rigid, k_rigid_b);
}

hipError_t tl_launch_p2g(const TlLaunch* L, int do_p2g, int tabs_differ, int cur, int rsb)
{
    KA_Args A;
    A.do_p2g = do_p2g;
    A.tabs_differ = tabs_differ;
    A.cur = cur;
    A.rsb = rsb;
    if (L->general)
        return tl_run_split(*L, k_p2g<1, false>, k_p2g_b<1, false>, k_p2g<1, true>, k_p2g_b<1, true>, A);
    return tl_run_split(*L, k_p2g<0, false>, k_p2g_b<0, false>, k_p2g<0, true>, k_p2g_b<0, true>, A);
}

hipError_t tl_launch_g2p(const TlLaunch* L, int cur)
{
    return tl_run_split(*L, k_g2p<false>, k_g2p_b<false>, k_g2p<true>, k_g2p_b<true>, cur);
}

hipError_t tl_launch_labels(const TlLaunch* L)
{
    if (L->S) { // one scene: TL_LBRICKS bricks per workgroup
        const int n = plain_bricks(*L);
        if (n <= 0) return hipSuccess;
        hipLaunchKernelGGL(k_labels_multi, dim3((n + TL_LBRICKS - 1) / TL_LBRICKS), dim3(256), 0, L->st, *L->S,
                           *L->D);
        return hipGetLastError();
    }
    const int n = L->n_items[IT_BRICK]; // a batch: TL_LBRICKS work items per workgroup
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_labels_multi_b, dim3((n + TL_LBRICKS - 1) / TL_LBRICKS), dim3(256), 0, L->st, L->Ks, L->Ds,
                       L->items[IT_BRICK], n);
    return hipGetLastError();
}

hipError_t tl_launch_labels_rigid(const TlLaunch* L)
{
    const int n = L->S ? plain_bricks(*L) : L->n_items[IT_BRICK];
    if (n <= 0) return hipSuccess;
    if (L->S)
        hipLaunchKernelGGL(k_labels_rigid, dim3(2 * n), dim3(256), 0, L->st, *L->S, *L->D, n);
    else
        hipLaunchKernelGGL(k_labels_rigid_b, dim3(2 * n), dim3(256), 0, L->st, L->Ks, L->Ds, L->items[IT_BRICK], n);
    return hipGetLastError();
}

hipError_t tl_launch_slots(const TlLaunch* L, int dst, int src, int force)
{
    return tl_run(*L, IT_NODE, plain_nodes(*L), 256, k_slots, k_slots_b, dst, src, force);
}

hipError_t tl_launch_mixed(const TlLaunch* L, int force)
{
    return tl_run(*L, IT_BRICK, plain_bricks(*L), 256, k_mixed, k_mixed_b, force);
}

hipError_t tl_launch_aabb(const TlLaunch* L)
{
    return tl_run(*L, IT_BRICK, plain_bricks(*L), 256, k_aabb, k_aabb_b);
}

hipError_t tl_launch_wrench(const TlLaunch* L)
{
    return tl_run(*L, IT_WRENCH, L->S ? TL_MAX_TOOLS * 6 : 0, 256, k_wrench, k_wrench_b);
}

hipError_t tl_launch_resetD(const TlLaunch* L)
{
    return tl_run(*L, IT_PART, plain_parts(*L), 256, k_resetD, k_resetD_b);
}

hipError_t tl_launch_call_start(const TlLaunch* L)
{
    return tl_run(*L, IT_SCENE, L->S ? 1 : 0, 64, k_call_start, k_call_start_b);
}

hipError_t tl_launch_fill_f32(float* p, long long n, float v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t tl_launch_fill_i32(int* p, long long n, int v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

// Device address of this GPU's copy of `scratch` (the batch workspace of
// tlmpm_batch_create_static), looked up once per device with that device current
// and kept: in host code the array's name is only a stand-in, never a device
// address.
hipError_t tl_static_scratch(int dev, void** ptr)
{
    static std::mutex m;
    static void* addr[TL_STATIC_DEVICES] = {};
    if (dev < 0 || dev >= TL_STATIC_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(m);
    if (!addr[dev]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != dev) return hipErrorInvalidDevice;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}
}
