// tlmpm_quad.hip -- gfx950 kernels of the quadratic B-spline variant of the
// transfers (27-node stencil, reading R33): P2G, grid update, G2P with the MUSL
// re-scatter, velocity remap and deformation-gradient update.  Labels, contact,
// cutting work and the wrench are shared with the trilinear path.
//
// A particle at reference coordinate q = (X - origin)/dx (in cells) touches the
// nodes base .. base + 2 per axis, base = floor(q - 1/2); a brick of 4x4x4 cells
// therefore touches the 7x7x7 box of nodes from (4 b - 1) to (4 b + 5).
//
// Logical grids (Sec. III-D) are slots of a per-node table of side keys, built each
// substep from the keys that reach the node: two tables alternate by substep
// parity, the table of one substep cleared during the next.
//
// Lanes.  Thread h * 64 + l of a brick workgroup holds, in each round, a particle
// of the brick's cell l whose position inside the cell has half pattern h (bit a
// set: upper half along axis a); the host builds this map once (reference
// positions do not move), with more rounds where a cell holds two particles of
// one pattern.  A wave's particles then lie in distinct cells with one pattern, so
// their base nodes, and the nodes of any one stencil offset, are distinct, and
// all of them lie in a 6x6x6 region fixed by the pattern.  For the brick's first
// side key each wave adds into its own LDS region with plain read-modify-writes
// (no atomics, no barriers); the regions are summed in wave order when the box
// goes out.  Further side keys of a brick (bricks on a cut) use LDS atomics, and
// beyond TL_QK keys HBM atomics.  The box sums go once per (node, slot) into HBM
// with floating-point atomics (up to 8 bricks share a node): results agree with
// the fixed-order trilinear path to rounding but are not bitwise reproducible.
#include <hip/hip_runtime.h>
#include <hip/amd_detail/amd_hip_unsafe_atomics.h>
#include <math.h>
#include <stdint.h>

#include "tlmpm_common.h"
#include "tlmpm_device.h"

#define TL_QBOX 7
#define TL_QBOXN 343      // nodes of a brick's 7x7x7 box
#define TL_QK 4           // side keys of a brick summed in LDS; further keys go to HBM directly
#define TL_QWG 512        // threads of a brick workgroup
#define TL_QEMPTY 0xFFFFFFFFu
#define TL_QREG 216       // nodes of one wave's 6x6x6 region (its 64 cells' stencils)

// brick-major id of grid node (gx, gy, gz); -1 outside the grid
DEV long long q_gid(const SceneK& S, int gx, int gy, int gz)
{
    if (gx < 0 || gy < 0 || gz < 0 || gx > S.cx || gy > S.cy || gz > S.cz) return -1;
    const long long nb = ((long long)(gz >> 2) * S.nby + (gy >> 2)) * S.nbx + (gx >> 2);
    return (nb << 6) | ((gz & 3) * 16 + (gy & 3) * 4 + (gx & 3));
}

// box node of a brick: (X, Y, Z) in 0..6 stands for grid node 4 b - 1 + (X, Y, Z)
DEV long long q_box_gid(const SceneK& S, int bx, int by, int bz, int bn)
{
    return q_gid(S, bx * TL_B - 1 + bn % TL_QBOX, by * TL_B - 1 + (bn / TL_QBOX) % TL_QBOX, bz * TL_B - 1 + bn / 49);
}

// grid cell of cell slot l (0..63, sorted order: parity class, cell) of brick (bx, by, bz)
DEV void q_cell(int bx, int by, int bz, int l, int c[3])
{
    const int w = l >> 3, i = l & 7;
    c[0] = bx * TL_B + 2 * (i & 1) + (w & 1);
    c[1] = by * TL_B + 2 * ((i >> 1) & 1) + ((w >> 1) & 1);
    c[2] = bz * TL_B + 2 * ((i >> 2) & 1) + ((w >> 2) & 1);
}

// Quadratic B-spline weights and derivatives per axis (reading R33).  The half of
// the cell the particle lies in (decided once on the host, in FP64) gives the base
// node; f = q - base lies in [1/2, 3/2) and the node distances are f, f - 1, f - 2:
//   N = (3/2 - f)^2 / 2,  3/4 - (f - 1)^2,  (f - 1/2)^2 / 2.
struct QStencil {
    int lo[3];        // base node per axis
    float w[3][3];    // [axis][node]
    float g[3][3];    // derivative / dx
};

DEV void q_stencil(const SceneK& S, const float* X, const int c[3], int h, QStencil& Q)
{
    const double o[3] = {S.ox, S.oy, S.oz};
#pragma unroll
    for (int a = 0; a < 3; a++) {
        double t = ((double)X[a] - o[a]) * S.inv_dx_d - (double)c[a];
        t = fmin(fmax(t, 0.0), 1.0);
        const bool low = ((h >> a) & 1) == 0; // the host's FP64 decision t < 1/2
        Q.lo[a] = low ? c[a] - 1 : c[a];
        const float f = (float)(low ? t + 1.0 : t);
        const float d0 = 1.5f - f, d1 = f - 1.0f, d2 = f - 0.5f;
        Q.w[a][0] = 0.5f * d0 * d0;
        Q.w[a][1] = 0.75f - d1 * d1;
        Q.w[a][2] = 0.5f * d2 * d2;
        Q.g[a][0] = -d0 * S.inv_dx;
        Q.g[a][1] = -2.0f * d1 * S.inv_dx;
        Q.g[a][2] = d2 * S.inv_dx;
    }
}

// index of a side key in the brick's LDS key list (inserted on first use); -1 full
DEV int q_key_index(uint32_t* s_keys, uint32_t key)
{
    for (int k = 0; k < TL_SCAP_MAX; k++) {
        const uint32_t old = atomicCAS(&s_keys[k], TL_QEMPTY, key);
        if (old == TL_QEMPTY || old == key) return k;
    }
    return -1;
}

// slot of key at node g in a table (slots fill from 0; the first empty one ends
// the list); -1 if absent
DEV int q_find(const SceneK& S, const uint32_t* tab, long long g, uint32_t key)
{
    for (int s = 0; s < S.scap; s++) {
        const uint32_t c = tab[(long long)s * S.NN + g];
        if (c == key) return s;
        if (c == TL_QEMPTY) return -1;
    }
    return -1;
}

DEV uint32_t* q_table(const SceneK& S, const SceneD& D, int par)
{
    return D.qcode + (size_t)par * (size_t)S.scap * (size_t)S.NN;
}

// Compatibility coupling of one 3-vector field over the c slots of a node (Eq. 8):
// f_a + (1/M) sum_{b != a, compatible} (m_a f_b - m_b f_a), M = sum of the masses,
// from the pre-exchange values; written over f.
DEV void q_couple(int c, const float* m, const uint32_t* codes, float (*f)[3])
{
    float M = 0.0f;
    for (int a = 0; a < c; a++) M += m[a];
    const float invM = M > 0.0f ? 1.0f / M : 0.0f;
    float out[TL_SCAP_MAX][3];
    for (int a = 0; a < c; a++) {
        float acc[3] = {0.0f, 0.0f, 0.0f};
        for (int b = 0; b < c; b++) {
            if (b == a || codes_conflict(codes[a], codes[b])) continue;
            for (int j = 0; j < 3; j++) acc[j] += m[a] * f[b][j] - m[b] * f[a][j];
        }
        for (int j = 0; j < 3; j++) out[a][j] = f[a][j] + acc[j] * invM;
    }
    for (int a = 0; a < c; a++)
        for (int j = 0; j < 3; j++) f[a][j] = out[a][j];
}

// particle of this thread in round r of active brick bi (-1: none)
DEV int q_particle(const SceneD& D, int bi, int r)
{
    return D.qmap[(size_t)(D.qround[bi] + r) * TL_QWG + threadIdx.x];
}

DEV int q_rounds(const SceneD& D, int bi) { return D.qround[bi + 1] - D.qround[bi]; }

// element i (0..2) of a 3-array by selects, so that a rolled loop keeps the array
// in registers
DEV float q_pick(const float (&a)[3], int i) { return i == 0 ? a[0] : (i == 1 ? a[1] : a[2]); }

// index of a key already in the brick's LDS key list; -1 if absent
DEV int q_key_lookup(const uint32_t* s_keys, uint32_t key)
{
    for (int k = 0; k < TL_SCAP_MAX; k++) {
        const uint32_t c = s_keys[k];
        if (c == key) return k;
        if (c == TL_QEMPTY) return -1;
    }
    return -1;
}

// registers the side keys of a brick's particles in its LDS key list (call between
// barriers)
DEV void q_register_keys(const SceneK& S, const SceneD& D, int bi, uint32_t* s_keys)
{
    const int rounds = q_rounds(D, bi);
    for (int r = 0; r < rounds; r++) {
        const int p = q_particle(D, bi, r);
        if (p < 0) continue;
        if (q_key_index(s_keys, slot_key(S, D.code[p])) < 0) atomicOr(D.status, TL_ST_BOX);
    }
}

// loads Q floats per node slot (from src, stride QS, offset off) for the first
// TL_QK keys of the brick over its box into dst[key][box node][Q]; absent slots
// read as zero
template <int Q, int QS, int OFF>
DEV void q_load_box(const SceneK& S, const uint32_t* tab, const float* src, int bx, int by, int bz,
                    const uint32_t* s_keys, float* dst)
{
    for (int t = threadIdx.x; t < TL_QK * TL_QBOXN; t += TL_QWG) {
        const uint32_t key = s_keys[t / TL_QBOXN];
        if (key == TL_QEMPTY) continue;
        const long long g = q_box_gid(S, bx, by, bz, t % TL_QBOXN);
        const int s = g >= 0 ? q_find(S, tab, g, key) : -1;
        float* o = dst + (size_t)t * Q;
        if (s < 0) {
#pragma unroll
            for (int c = 0; c < Q; c++) o[c] = 0.0f;
            continue;
        }
        const float* a = src + ((size_t)g * S.scap + s) * QS + OFF;
#pragma unroll
        for (int c = 0; c < Q; c++) o[c] = a[c];
    }
}

// ------------------------------------------------------------------ slot tables
// Per active brick: clears the other parity's table over its box, then inserts the
// side key of every (box node, key) reached by a particle with a non-zero weight
// into this parity's table (atomic compare-and-swap per slot); a new slot's sums
// are zeroed by the thread that created it.
__global__ __launch_bounds__(TL_QWG) void k_q_slots(SceneK S, SceneD D, int par)
{
    __shared__ uint32_t s_keys[TL_SCAP_MAX];
    __shared__ uint32_t s_pres[TL_QBOXN];
    const int bi = blockIdx.x, tid = threadIdx.x;
    const int brick = D.active[bi];
    const int bx = brick % S.cbx, by = (brick / S.cbx) % S.cby, bz = brick / (S.cbx * S.cby);
    uint32_t* tab = q_table(S, D, par);
    uint32_t* other = q_table(S, D, 1 - par);
    for (int t = tid; t < TL_QBOXN; t += TL_QWG) {
        s_pres[t] = 0u;
        const long long g = q_box_gid(S, bx, by, bz, t);
        if (g < 0) continue;
        for (int s = 0; s < S.scap; s++) {
            const long long i = (long long)s * S.NN + g;
            if (other[i] == TL_QEMPTY) break;
            other[i] = TL_QEMPTY;
        }
    }
    if (tid < TL_SCAP_MAX) s_keys[tid] = TL_QEMPTY;
    __syncthreads();
    const long long N = S.N;
    const int rounds = q_rounds(D, bi), h = tid >> 6;
    int c[3];
    q_cell(bx, by, bz, tid & 63, c);
    for (int r = 0; r < rounds; r++) {
        const int p = q_particle(D, bi, r);
        if (p < 0) continue;
        const uint32_t key = slot_key(S, D.code[p]);
        const int k = q_key_index(s_keys, key);
        if (k < 0) {
            atomicOr(D.status, TL_ST_BOX);
            continue;
        }
        const float X[3] = {D.X[p], D.X[N + p], D.X[2 * N + p]};
        QStencil Q;
        q_stencil(S, X, c, h, Q);
        const int ox = Q.lo[0] - (bx * TL_B - 1), oy = Q.lo[1] - (by * TL_B - 1), oz = Q.lo[2] - (bz * TL_B - 1);
#pragma unroll
        for (int cz = 0; cz < 3; cz++)
#pragma unroll
            for (int cy = 0; cy < 3; cy++)
#pragma unroll
                for (int cx = 0; cx < 3; cx++) {
                    if (Q.w[0][cx] * Q.w[1][cy] * Q.w[2][cz] == 0.0f) continue; // reading R7
                    atomicOr(&s_pres[((oz + cz) * TL_QBOX + oy + cy) * TL_QBOX + ox + cx], 1u << k);
                }
    }
    __syncthreads();
    for (int t = tid; t < TL_QBOXN; t += TL_QWG) {
        uint32_t pm = s_pres[t];
        if (!pm) continue;
        const long long g = q_box_gid(S, bx, by, bz, t);
        if (g < 0) {
            atomicOr(D.status, TL_ST_BOX);
            continue;
        }
        while (pm) {
            const int k = __ffs(pm) - 1;
            pm &= pm - 1u;
            const uint32_t key = s_keys[k];
            int s = 0;
            for (; s < S.scap; s++) {
                const uint32_t old = atomicCAS(&tab[(long long)s * S.NN + g], TL_QEMPTY, key);
                if (old == TL_QEMPTY) {
                    float4* a = (float4*)(D.qacc + ((size_t)g * S.scap + s) * 8);
                    a[0] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    a[1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    *(float4*)(D.qrs + ((size_t)g * S.scap + s) * 4) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    break;
                }
                if (old == key) break;
            }
            if (s == S.scap) atomicOr(D.status, TL_ST_SLOT);
        }
    }
}

// adds a brick's LDS sums (Q values per node) into the node slots in HBM (stride
// QS floats per slot): the first key's sums from the 8 wave regions, in wave order
// (wave h holds box node (X, Y, Z) at region (X, Y, Z) - 1 + low(h), low = 1 on the
// axes of the lower half), the other keys' sums from s_acc [key - 1][box node]
template <int Q, int QS>
DEV void q_flush(const SceneK& S, const SceneD& D, const uint32_t* tab, float* dst, int bx, int by, int bz,
                 const uint32_t* s_keys, const float* s_wv, const float* s_acc)
{
    for (int t = threadIdx.x; t < TL_QK * TL_QBOXN; t += TL_QWG) {
        const int k = t / TL_QBOXN, bn = t % TL_QBOXN;
        const uint32_t key = s_keys[k];
        if (key == TL_QEMPTY) continue;
        float v[Q];
        if (k == 0) {
            const int X = bn % TL_QBOX, Y = (bn / TL_QBOX) % TL_QBOX, Z = bn / 49;
#pragma unroll
            for (int c = 0; c < Q; c++) v[c] = 0.0f;
#pragma unroll
            for (int h = 0; h < 8; h++) {
                const int rx = X - (h & 1), ry = Y - ((h >> 1) & 1), rz = Z - ((h >> 2) & 1);
                if (rx < 0 || ry < 0 || rz < 0 || rx > 5 || ry > 5 || rz > 5) continue;
                const float* w = s_wv + ((size_t)h * TL_QREG + (rz * 6 + ry) * 6 + rx) * Q;
#pragma unroll
                for (int c = 0; c < Q; c++) v[c] += w[c];
            }
        } else {
#pragma unroll
            for (int c = 0; c < Q; c++) v[c] = s_acc[((size_t)(k - 1) * TL_QBOXN + bn) * Q + c];
        }
        bool any = false;
#pragma unroll
        for (int c = 0; c < Q; c++) any = any || v[c] != 0.0f;
        if (!any) continue;
        const long long g = q_box_gid(S, bx, by, bz, bn);
        const int s = g >= 0 ? q_find(S, tab, g, key) : -1;
        if (s < 0) {
            atomicOr(D.status, TL_ST_LOOKUP);
            continue;
        }
        float* o = dst + ((size_t)g * S.scap + s) * QS;
#pragma unroll
        for (int c = 0; c < Q; c++)
            if (v[c] != 0.0f) unsafeAtomicAdd(o + c, v[c]);
    }
}

// ---------------------------------------------------------------------------- P2G
// Per active brick: stress (Neo-Hookean, or the fixed-corotated family with
// viscosity and plasticity for MAT 1), gravity and contact impulses, and the
// label-masked scatter of m, m v and the impulse (Eq. 2) to the 27 nodes.
template <int MAT>
__global__ __launch_bounds__(TL_QWG) void k_q_p2g(SceneK S, SceneD D, int par)
{
    __shared__ uint32_t s_keys[TL_SCAP_MAX];
    __shared__ float s_wv[8 * TL_QREG * 7];
    __shared__ float s_acc[(TL_QK - 1) * TL_QBOXN * 7];
    const int bi = blockIdx.x, tid = threadIdx.x;
    const int brick = D.active[bi];
    const int bx = brick % S.cbx, by = (brick / S.cbx) % S.cby, bz = brick / (S.cbx * S.cby);
    const uint32_t* tab = q_table(S, D, par);
    for (int t = tid; t < 8 * TL_QREG * 7; t += TL_QWG) s_wv[t] = 0.0f;
    for (int t = tid; t < (TL_QK - 1) * TL_QBOXN * 7; t += TL_QWG) s_acc[t] = 0.0f;
    if (tid < TL_SCAP_MAX) s_keys[tid] = TL_QEMPTY;
    __syncthreads();
    const long long N = S.N;
    const float dt = S.dt;
    const bool rig = (S.floor_on || D.tinfo[1]) && D.brig[brick] != 0;
    const int rounds = q_rounds(D, bi), h = tid >> 6;
    int c[3];
    q_cell(bx, by, bz, tid & 63, c);
    for (int r = 0; r < rounds; r++) {
        const int p = q_particle(D, bi, r);
        bool valid = p >= 0;
        int k = -1;
        uint32_t key = 0;
        float m = 0.0f, vel[3] = {0.0f, 0.0f, 0.0f}, ext[3] = {0.0f, 0.0f, 0.0f};
        float Pk[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        QStencil Q = {};
        if (valid) {
            const uint32_t code = D.code[p];
            key = slot_key(S, code);
            k = q_key_index(s_keys, key);
            if (k < 0) atomicOr(D.status, TL_ST_BOX);
            valid = k >= 0;
        }
        if (valid) {
            float H[9];
            const uint32_t code = D.code[p];
            const float X[3] = {D.X[p], D.X[N + p], D.X[2 * N + p]};
#pragma unroll
            for (int a = 0; a < 9; a++) H[a] = D.H[a * N + p];
#pragma unroll
            for (int a = 0; a < 3; a++) vel[a] = D.v[a * N + p];
            m = S.m_uniform ? S.m0 : D.m[p];
            const float V0 = S.v_uniform ? S.V0 : D.V0[p];
            const float E = S.e_uniform ? S.E0 : D.E[p];
            bool ok;
            if constexpr (MAT == 1) {
                if (S.ystress > 0.0f) {
                    // P = P_fcr(F_e) F_p^{-T}, F_e - I = H + Gp + H Gp, F_p^{-1} = I + Gp
                    float Gp[9], K[9], Pe[9];
#pragma unroll
                    for (int a = 0; a < 9; a++) Gp[a] = D.Gp[a * N + p];
#pragma unroll
                    for (int i = 0; i < 3; i++)
#pragma unroll
                        for (int j = 0; j < 3; j++) {
                            float kk = H[3 * i + j] + Gp[3 * i + j];
#pragma unroll
                            for (int l = 0; l < 3; l++) kk += H[3 * i + l] * Gp[3 * l + j];
                            K[3 * i + j] = kk;
                        }
                    ok = fixed_corotated(E, S.nu, K, Pe);
#pragma unroll
                    for (int i = 0; i < 3; i++)
#pragma unroll
                        for (int j = 0; j < 3; j++) {
                            float a = Pe[3 * i + j];
#pragma unroll
                            for (int l = 0; l < 3; l++) a += Pe[3 * i + l] * Gp[3 * j + l];
                            Pk[3 * i + j] = a;
                        }
                } else {
                    ok = S.material == 1 ? fixed_corotated(E, S.nu, H, Pk) : neo_hookean(E, S.nu, H, Pk);
                }
                if (ok && S.visc > 0.0f) {
                    float Fd[9];
#pragma unroll
                    for (int a = 0; a < 9; a++) Fd[a] = D.Fdot[a * N + p];
                    add_viscous(S.visc, H, Fd, Pk);
                }
            } else {
                ok = neo_hookean(E, S.nu, H, Pk);
            }
            if (!ok) {
                atomicOr(D.status, TL_ST_NONFINITE);
#pragma unroll
                for (int a = 0; a < 9; a++) Pk[a] = 0.0f;
            }
            float Jc[3] = {0.0f, 0.0f, 0.0f};
            if (rig) {
                Jc[0] += D.Jrig[p];
                Jc[1] += D.Jrig[N + p];
                Jc[2] += D.Jrig[2 * N + p];
            }
            if (S.material_contact && (code & TL_CAND_BIT)) {
                Jc[0] += D.Jmat[p];
                Jc[1] += D.Jmat[N + p];
                Jc[2] += D.Jmat[2 * N + p];
            }
#pragma unroll
            for (int a = 0; a < 3; a++) ext[a] = Jc[a] + dt * m * (a == 0 ? S.gx : a == 1 ? S.gy : S.gz);
            const float sA = -dt * V0;
#pragma unroll
            for (int a = 0; a < 9; a++) Pk[a] *= sA;
            q_stencil(S, X, c, h, Q);
        }
        const int ox = Q.lo[0] - (bx * TL_B - 1), oy = Q.lo[1] - (by * TL_B - 1), oz = Q.lo[2] - (bz * TL_B - 1);
        // the 7 sums of node (cx, cy, cz): m, m v, and the impulse A grad N + w ext
        auto node_vals = [&](int cx, int cy, int cz, float* val) {
            const float wx = q_pick(Q.w[0], cx), wy = q_pick(Q.w[1], cy), wz = q_pick(Q.w[2], cz);
            const float w = wx * wy * wz;
            const float g0 = q_pick(Q.g[0], cx) * wy * wz;
            const float g1 = wx * q_pick(Q.g[1], cy) * wz;
            const float g2 = wx * wy * q_pick(Q.g[2], cz);
            val[0] = w * m;
            val[1] = val[0] * vel[0];
            val[2] = val[0] * vel[1];
            val[3] = val[0] * vel[2];
#pragma unroll
            for (int a = 0; a < 3; a++) val[4 + a] = Pk[3 * a] * g0 + Pk[3 * a + 1] * g1 + Pk[3 * a + 2] * g2 + w * ext[a];
            return w != 0.0f; // reading R7: a zero weight contributes nothing
        };
        if (valid && k >= TL_QK) {
            // more side keys in this brick than LDS holds: straight to the node slots
#pragma unroll 1
            for (int t = 0; t < 27; t++) {
                const int cx = t % 3, cy = (t / 3) % 3, cz = t / 9;
                float val[7];
                if (!node_vals(cx, cy, cz, val)) continue;
                const long long g = q_gid(S, Q.lo[0] + cx, Q.lo[1] + cy, Q.lo[2] + cz);
                const int s = g >= 0 ? q_find(S, tab, g, key) : -1;
                if (s < 0) {
                    atomicOr(D.status, TL_ST_LOOKUP);
                    continue;
                }
                float* o = D.qacc + ((size_t)g * S.scap + s) * 8;
#pragma unroll
                for (int q = 0; q < 7; q++) unsafeAtomicAdd(o + q, val[q]);
            }
        }
        if (valid && k == 0) {
            // own region of this wave: the lanes' nodes of one offset are distinct
            const int rx = c[0] - bx * TL_B, ry = c[1] - by * TL_B, rz = c[2] - bz * TL_B;
            float* d0 = s_wv + (size_t)h * TL_QREG * 7;
#pragma unroll
            for (int cz = 0; cz < 3; cz++)
#pragma unroll
                for (int cy = 0; cy < 3; cy++) {
#pragma unroll
                    for (int cx = 0; cx < 3; cx++) {
                        float val[7];
                        if (!node_vals(cx, cy, cz, val)) continue;
                        float* d = d0 + (((rz + cz) * 6 + ry + cy) * 6 + rx + cx) * 7;
#pragma unroll
                        for (int q = 0; q < 7; q++) d[q] += val[q];
                    }
                    // one row of nodes at a time: keeps the compiler from hoisting all
                    // 189 reads (and their registers) to the top
                    asm volatile("" ::: "memory");
                }
        } else if (valid && k < TL_QK) {
            float* d0 = s_acc + (size_t)(k - 1) * TL_QBOXN * 7;
#pragma unroll 1
            for (int t = 0; t < 27; t++) {
                const int cx = t % 3, cy = (t / 3) % 3, cz = t / 9;
                float val[7];
                if (!node_vals(cx, cy, cz, val)) continue;
                float* d = d0 + (((oz + cz) * TL_QBOX + oy + cy) * TL_QBOX + ox + cx) * 7;
#pragma unroll
                for (int q = 0; q < 7; q++) atomicAdd(d + q, val[q]);
            }
        }
    }
    __syncthreads();
    q_flush<7, 8>(S, D, tab, D.qacc, bx, by, bz, s_keys, s_wv, s_acc);
}

// ---------------------------------------------------------------- node kernels
// Grid update: per node, coupling of momentum and impulse (Eq. 8), then
// v^n = pbar / m and dv = dpbar / m (Eq. 9) over the slot's sums.
__global__ __launch_bounds__(256) void k_q_grid(SceneK S, SceneD D, int par)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= D.n_qnodes) return;
    const long long g = D.qnodes[i];
    const uint32_t* tab = q_table(S, D, par);
    uint32_t codes[TL_SCAP_MAX];
    int c = 0;
    for (; c < S.scap; c++) {
        codes[c] = tab[(long long)c * S.NN + g];
        if (codes[c] == TL_QEMPTY) break;
    }
    if (c == 0) return;
    float* a = D.qacc + (size_t)g * S.scap * 8;
    if (c == 1) {
        const float m = a[0], im = m > 0.0f ? 1.0f / m : 0.0f;
        for (int j = 1; j < 7; j++) a[j] *= im;
        return;
    }
    float m[TL_SCAP_MAX], p[TL_SCAP_MAX][3], dp[TL_SCAP_MAX][3];
    for (int s = 0; s < c; s++) {
        m[s] = a[s * 8];
        for (int j = 0; j < 3; j++) {
            p[s][j] = a[s * 8 + 1 + j];
            dp[s][j] = a[s * 8 + 4 + j];
        }
    }
    q_couple(c, m, codes, p);
    q_couple(c, m, codes, dp);
    for (int s = 0; s < c; s++) {
        const float im = m[s] > 0.0f ? 1.0f / m[s] : 0.0f;
        for (int j = 0; j < 3; j++) {
            a[s * 8 + 1 + j] = p[s][j] * im;
            a[s * 8 + 4 + j] = dp[s][j] * im;
        }
    }
}

// Velocity remap of the MUSL re-scatter: per node, coupling of m v^{n+1} (Eq. 8),
// then v~ = ptbar / m.
__global__ __launch_bounds__(256) void k_q_remap(SceneK S, SceneD D, int par)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= D.n_qnodes) return;
    const long long g = D.qnodes[i];
    const uint32_t* tab = q_table(S, D, par);
    uint32_t codes[TL_SCAP_MAX];
    int c = 0;
    for (; c < S.scap; c++) {
        codes[c] = tab[(long long)c * S.NN + g];
        if (codes[c] == TL_QEMPTY) break;
    }
    if (c == 0) return;
    const float* a = D.qacc + (size_t)g * S.scap * 8;
    float* r = D.qrs + (size_t)g * S.scap * 4;
    if (c == 1) {
        const float m = a[0], im = m > 0.0f ? 1.0f / m : 0.0f;
        for (int j = 0; j < 3; j++) r[j] *= im;
        return;
    }
    float m[TL_SCAP_MAX], pt[TL_SCAP_MAX][3];
    for (int s = 0; s < c; s++) {
        m[s] = a[s * 8];
        for (int j = 0; j < 3; j++) pt[s][j] = r[s * 4 + j];
    }
    q_couple(c, m, codes, pt);
    for (int s = 0; s < c; s++) {
        const float im = m[s] > 0.0f ? 1.0f / m[s] : 0.0f;
        for (int j = 0; j < 3; j++) r[s * 4 + j] = pt[s][j] * im;
    }
}

// ---------------------------------------------------------------------------- G2P
// Per active brick: the box's grid velocities (v^n, dv) of its first TL_QK side
// keys into LDS, PIC/FLIP update of v and x (Eq. 17), the MUSL re-scatter of
// m_p v_p^{n+1}, and the brick's AABB and speed bound.
__global__ __launch_bounds__(TL_QWG) void k_q_g2p(SceneK S, SceneD D, int par)
{
    __shared__ uint32_t s_keys[TL_SCAP_MAX];
    __shared__ float s_grid[TL_QK * TL_QBOXN * 6];
    __shared__ float s_wv[8 * TL_QREG * 3];
    __shared__ float s_acc[(TL_QK - 1) * TL_QBOXN * 3];
    __shared__ float s_bb[TL_QWG / 64][7];
    const int bi = blockIdx.x, tid = threadIdx.x;
    const int brick = D.active[bi];
    if (bi == 0 && tid == 0) {
        // end of the substep for this scene: next history stamp and substep index
        // (no later kernel of the substep reads them)
        D.ctr[0] += 1;
        D.ctr[2] += 1;
    }
    const int bx = brick % S.cbx, by = (brick / S.cbx) % S.cby, bz = brick / (S.cbx * S.cby);
    const uint32_t* tab = q_table(S, D, par);
    for (int t = tid; t < 8 * TL_QREG * 3; t += TL_QWG) s_wv[t] = 0.0f;
    for (int t = tid; t < (TL_QK - 1) * TL_QBOXN * 3; t += TL_QWG) s_acc[t] = 0.0f;
    if (tid < TL_SCAP_MAX) s_keys[tid] = TL_QEMPTY;
    __syncthreads();
    q_register_keys(S, D, bi, s_keys);
    __syncthreads();
    q_load_box<6, 8, 1>(S, tab, D.qacc, bx, by, bz, s_keys, s_grid);
    __syncthreads();
    const long long N = S.N;
    const float dt = S.dt, beta = S.beta;
    const int rounds = q_rounds(D, bi), h = tid >> 6;
    int c[3];
    q_cell(bx, by, bz, tid & 63, c);
    float bb[7] = {1e30f, 1e30f, 1e30f, -1e30f, -1e30f, -1e30f, 0.0f};
    for (int r = 0; r < rounds; r++) {
        const int p = q_particle(D, bi, r);
        int k = -1;
        uint32_t key = 0;
        if (p >= 0) {
            key = slot_key(S, D.code[p]);
            k = q_key_lookup(s_keys, key); // -1 was flagged when the keys were registered
        }
        const bool valid = k >= 0;
        float m = 0.0f, vn1[3] = {0.0f, 0.0f, 0.0f};
        QStencil Q = {};
        if (valid) {
            const float X[3] = {D.X[p], D.X[N + p], D.X[2 * N + p]};
            q_stencil(S, X, c, h, Q);
            float av[3] = {0.0f, 0.0f, 0.0f}, ax[3] = {0.0f, 0.0f, 0.0f};
            auto add_node = [&](float w, const float* vn, const float* dv) {
#pragma unroll
                for (int j = 0; j < 3; j++) {
                    av[j] += w * ((1.0f - beta) * vn[j] + dv[j]);
                    ax[j] += w * (vn[j] + dv[j]);
                }
            };
            if (k < TL_QK) {
                const int ox = Q.lo[0] - (bx * TL_B - 1), oy = Q.lo[1] - (by * TL_B - 1), oz = Q.lo[2] - (bz * TL_B - 1);
                const float* g0 = s_grid + (size_t)k * TL_QBOXN * 6;
#pragma unroll
                for (int cz = 0; cz < 3; cz++)
#pragma unroll
                    for (int cy = 0; cy < 3; cy++)
#pragma unroll
                        for (int cx = 0; cx < 3; cx++) {
                            const float w = Q.w[0][cx] * Q.w[1][cy] * Q.w[2][cz];
                            if (w == 0.0f) continue;
                            const float* a = g0 + (((oz + cz) * TL_QBOX + oy + cy) * TL_QBOX + ox + cx) * 6;
                            add_node(w, a, a + 3);
                        }
            } else {
#pragma unroll 1
                for (int t = 0; t < 27; t++) {
                    const int cx = t % 3, cy = (t / 3) % 3, cz = t / 9;
                    const float w = q_pick(Q.w[0], cx) * q_pick(Q.w[1], cy) * q_pick(Q.w[2], cz);
                    if (w == 0.0f) continue;
                    const long long g = q_gid(S, Q.lo[0] + cx, Q.lo[1] + cy, Q.lo[2] + cz);
                    const int s = g >= 0 ? q_find(S, tab, g, key) : -1;
                    if (s < 0) {
                        atomicOr(D.status, TL_ST_LOOKUP);
                        continue;
                    }
                    const float* a = D.qacc + ((size_t)g * S.scap + s) * 8;
                    add_node(w, a + 1, a + 4);
                }
            }
#pragma unroll
            for (int j = 0; j < 3; j++) {
                vn1[j] = beta * D.v[j * N + p] + av[j];
                const float un = D.u[j * N + p] + dt * ax[j];
                D.v[j * N + p] = vn1[j];
                D.u[j * N + p] = un;
                const float xa = X[j] + un;
                bb[j] = fminf(bb[j], xa);
                bb[3 + j] = fmaxf(bb[3 + j], xa);
            }
            bb[6] = fmaxf(bb[6], sqrtf(vn1[0] * vn1[0] + vn1[1] * vn1[1] + vn1[2] * vn1[2]));
            m = S.m_uniform ? S.m0 : D.m[p];
        }
        if (valid && k >= TL_QK) {
#pragma unroll 1
            for (int t = 0; t < 27; t++) {
                const int cx = t % 3, cy = (t / 3) % 3, cz = t / 9;
                const float wm = q_pick(Q.w[0], cx) * q_pick(Q.w[1], cy) * q_pick(Q.w[2], cz) * m;
                if (wm == 0.0f) continue;
                const long long g = q_gid(S, Q.lo[0] + cx, Q.lo[1] + cy, Q.lo[2] + cz);
                const int s = g >= 0 ? q_find(S, tab, g, key) : -1;
                if (s < 0) {
                    atomicOr(D.status, TL_ST_LOOKUP);
                    continue;
                }
                float* o = D.qrs + ((size_t)g * S.scap + s) * 4;
#pragma unroll
                for (int j = 0; j < 3; j++) unsafeAtomicAdd(o + j, wm * vn1[j]);
            }
        }
        // MUSL re-scatter of m v^{n+1} (wave regions as in the P2G)
        if (valid && k == 0) {
            const int rx = c[0] - bx * TL_B, ry = c[1] - by * TL_B, rz = c[2] - bz * TL_B;
            float* d0 = s_wv + (size_t)h * TL_QREG * 3;
#pragma unroll
            for (int cz = 0; cz < 3; cz++)
#pragma unroll
                for (int cy = 0; cy < 3; cy++)
#pragma unroll
                    for (int cx = 0; cx < 3; cx++) {
                        const float wm = Q.w[0][cx] * Q.w[1][cy] * Q.w[2][cz] * m;
                        if (wm == 0.0f) continue;
                        float* d = d0 + (((rz + cz) * 6 + ry + cy) * 6 + rx + cx) * 3;
#pragma unroll
                        for (int j = 0; j < 3; j++) d[j] += wm * vn1[j];
                    }
        } else if (valid && k < TL_QK) {
            const int ox = Q.lo[0] - (bx * TL_B - 1), oy = Q.lo[1] - (by * TL_B - 1), oz = Q.lo[2] - (bz * TL_B - 1);
            float* d0 = s_acc + (size_t)(k - 1) * TL_QBOXN * 3;
#pragma unroll 1
            for (int t = 0; t < 27; t++) {
                const int cx = t % 3, cy = (t / 3) % 3, cz = t / 9;
                const float wm = q_pick(Q.w[0], cx) * q_pick(Q.w[1], cy) * q_pick(Q.w[2], cz) * m;
                if (wm == 0.0f) continue;
                float* d = d0 + (((oz + cz) * TL_QBOX + oy + cy) * TL_QBOX + ox + cx) * 3;
#pragma unroll
                for (int j = 0; j < 3; j++) atomicAdd(d + j, wm * vn1[j]);
            }
        }
    }
    // brick AABB of x^{n+1} and speed bound (used to skip distant contact work)
    const int lane = tid & 63, wv = tid >> 6;
    for (int q = 0; q < 7; q++) {
        float val = bb[q];
        for (int o = 1; o < 64; o <<= 1) {
            const float other = __shfl_xor(val, o, 64);
            val = (q < 3) ? fminf(val, other) : fmaxf(val, other);
        }
        if (lane == 0) s_bb[wv][q] = val;
    }
    __syncthreads();
    if (tid < 7) {
        float val = s_bb[0][tid];
        for (int w = 1; w < TL_QWG / 64; w++) val = (tid < 3) ? fminf(val, s_bb[w][tid]) : fmaxf(val, s_bb[w][tid]);
        D.aabb[(long long)brick * 8 + tid] = val;
        if (tid == 6 && S.material_contact && val > 0.0f)
            atomicMax(D.hmax + (bi & (TL_HSLOTS - 1)) * TL_HSTRIDE, __float_as_int(val));
    }
    q_flush<3, 4>(S, D, tab, D.qrs, bx, by, bz, s_keys, s_wv, s_acc);
}

// --------------------------------------------------------------- F update (MUSL)
// Per active brick: the box's remapped velocities of its first TL_QK side keys into
// LDS, then per particle F += dt sum_i v~_i (x) grad N_i with its own slots; the
// rate is kept for viscosity and the plastic projection follows (MAT 1).
template <int MAT>
__global__ __launch_bounds__(TL_QWG) void k_q_F(SceneK S, SceneD D, int par)
{
    __shared__ uint32_t s_keys[TL_SCAP_MAX];
    __shared__ float s_vt[TL_QK * TL_QBOXN * 3];
    const int bi = blockIdx.x, tid = threadIdx.x;
    const int brick = D.active[bi];
    const int bx = brick % S.cbx, by = (brick / S.cbx) % S.cby, bz = brick / (S.cbx * S.cby);
    const uint32_t* tab = q_table(S, D, par);
    if (tid < TL_SCAP_MAX) s_keys[tid] = TL_QEMPTY;
    __syncthreads();
    q_register_keys(S, D, bi, s_keys);
    __syncthreads();
    q_load_box<3, 4, 0>(S, tab, D.qrs, bx, by, bz, s_keys, s_vt);
    __syncthreads();
    const long long N = S.N;
    const float dt = S.dt;
    const int rounds = q_rounds(D, bi), h = tid >> 6;
    int c[3];
    q_cell(bx, by, bz, tid & 63, c);
    for (int r = 0; r < rounds; r++) {
        const int p = q_particle(D, bi, r);
        if (p < 0) continue;
        const uint32_t key = slot_key(S, D.code[p]);
        const int k = q_key_lookup(s_keys, key);
        if (k < 0) continue;
        const float X[3] = {D.X[p], D.X[N + p], D.X[2 * N + p]};
        QStencil Q;
        q_stencil(S, X, c, h, Q);
        float Lg[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        auto add_node = [&](float g0, float g1, float g2, const float* v) {
#pragma unroll
            for (int a = 0; a < 3; a++) {
                Lg[3 * a + 0] += v[a] * g0;
                Lg[3 * a + 1] += v[a] * g1;
                Lg[3 * a + 2] += v[a] * g2;
            }
        };
        if (k < TL_QK) {
            const int ox = Q.lo[0] - (bx * TL_B - 1), oy = Q.lo[1] - (by * TL_B - 1), oz = Q.lo[2] - (bz * TL_B - 1);
            const float* v0 = s_vt + (size_t)k * TL_QBOXN * 3;
#pragma unroll
            for (int cz = 0; cz < 3; cz++)
#pragma unroll
                for (int cy = 0; cy < 3; cy++)
#pragma unroll
                    for (int cx = 0; cx < 3; cx++) {
                        if (Q.w[0][cx] * Q.w[1][cy] * Q.w[2][cz] == 0.0f) continue;
                        add_node(Q.g[0][cx] * Q.w[1][cy] * Q.w[2][cz], Q.w[0][cx] * Q.g[1][cy] * Q.w[2][cz],
                                 Q.w[0][cx] * Q.w[1][cy] * Q.g[2][cz],
                                 v0 + (((oz + cz) * TL_QBOX + oy + cy) * TL_QBOX + ox + cx) * 3);
                    }
        } else {
#pragma unroll 1
            for (int t = 0; t < 27; t++) {
                const int cx = t % 3, cy = (t / 3) % 3, cz = t / 9;
                const float wx = q_pick(Q.w[0], cx), wy = q_pick(Q.w[1], cy), wz = q_pick(Q.w[2], cz);
                if (wx * wy * wz == 0.0f) continue;
                const long long g = q_gid(S, Q.lo[0] + cx, Q.lo[1] + cy, Q.lo[2] + cz);
                const int s = g >= 0 ? q_find(S, tab, g, key) : -1;
                if (s < 0) {
                    atomicOr(D.status, TL_ST_LOOKUP);
                    continue;
                }
                add_node(q_pick(Q.g[0], cx) * wy * wz, wx * q_pick(Q.g[1], cy) * wz, wx * wy * q_pick(Q.g[2], cz),
                         D.qrs + ((size_t)g * S.scap + s) * 4);
            }
        }
        float H[9];
        bool fin = true;
#pragma unroll
        for (int a = 0; a < 9; a++) {
            H[a] = D.H[a * N + p] + dt * Lg[a];
            D.H[a * N + p] = H[a];
            fin = fin && isfinite(H[a]);
        }
        if (!fin) atomicOr(D.status, TL_ST_NONFINITE);
        if constexpr (MAT == 1) {
            if (S.visc > 0.0f)
#pragma unroll
                for (int a = 0; a < 9; a++) D.Fdot[a * N + p] = Lg[a];
            if (S.ystress > 0.0f) {
                float Gp[9], K[9];
#pragma unroll
                for (int a = 0; a < 9; a++) Gp[a] = D.Gp[a * N + p];
#pragma unroll
                for (int i = 0; i < 3; i++)
#pragma unroll
                    for (int j = 0; j < 3; j++) {
                        float kk = H[3 * i + j] + Gp[3 * i + j];
#pragma unroll
                        for (int l = 0; l < 3; l++) kk += H[3 * i + l] * Gp[3 * l + j];
                        K[3 * i + j] = kk;
                    }
                const float E = S.e_uniform ? S.E0 : D.E[p];
                if (vm_project(E, S.nu, S.ystress, K, Gp))
#pragma unroll
                    for (int a = 0; a < 9; a++) D.Gp[a * N + p] = Gp[a];
            }
        }
    }
}

// ------------------------------------------------------------------ host launches
extern "C" {

// the transfers of one substep of a single scene with the quadratic stencil, in
// order, with the table of parity par; timing class per launch via the callback
hipError_t tl_launch_quad(const TlLaunch* L, int par, int stage)
{
    const SceneK& S = *L->S;
    const SceneD& D = *L->D;
    const int nb = D.n_active;
    const int nn = (D.n_qnodes + 255) / 256;
    if (nb == 0) return hipSuccess;
    switch (stage) {
    case 0:
        k_q_slots<<<nb, TL_QWG, 0, L->st>>>(S, D, par);
        break;
    case 1:
        if (L->general)
            k_q_p2g<1><<<nb, TL_QWG, 0, L->st>>>(S, D, par);
        else
            k_q_p2g<0><<<nb, TL_QWG, 0, L->st>>>(S, D, par);
        break;
    case 2:
        if (nn) k_q_grid<<<nn, 256, 0, L->st>>>(S, D, par);
        break;
    case 3:
        k_q_g2p<<<nb, TL_QWG, 0, L->st>>>(S, D, par);
        break;
    case 4:
        if (nn) k_q_remap<<<nn, 256, 0, L->st>>>(S, D, par);
        break;
    case 5:
        if (L->general)
            k_q_F<1><<<nb, TL_QWG, 0, L->st>>>(S, D, par);
        else
            k_q_F<0><<<nb, TL_QWG, 0, L->st>>>(S, D, par);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

} // extern "C"
