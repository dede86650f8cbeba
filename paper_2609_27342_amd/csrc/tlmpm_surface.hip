// tlmpm_surface.hip -- surface reconstruction on the reference grid (Sec. III-F):
// the linked volume of the scene's current side codes, local dual contouring, and
// the one-way embedding of the surface in the particles' motion.  Visual output
// only: it runs on request, outside the substep.
//
// Lattice: the 2x2x2 sub-cell sites of the reference grid (spacing h = dx / 2),
// site s = floor((X - origin) / h) per axis; a site is material when a particle
// lies in it (the particle of smallest caller index if several do).  A link
// between face-adjacent sites is intact when both are material and their side
// codes do not conflict (the blade sweep that gave them opposite digits cut it);
// a directed link from a material site is a transition otherwise.  Each cube of
// 8 sites splits its material corners into regions, the connected components of
// its intact edges; a region with a transition edge gets one vertex, placed per
// axis at the mean coordinate of its transition-link midpoints along that axis
// (along all of them when it has none: the minimiser of the quadratic error of
// Hermite planes whose normals are the link directions).  Each directed
// transition gives one quad through the vertices of its site's regions in the
// four cubes around the link, counter-clockwise about the outward direction; a
// cut link gives one quad per side, the two coincident faces of the cut.  A
// vertex moves with fixed trilinear weights over its region's particles.
//
// Workspace (caller's, see tlmpm_surface_build): site table u64 [S] (caller index
// << 32 | sorted index, ~0 empty), cube region map u32 [C] (4 bits per corner: the
// corner's vertex among the cube's, 0xE material without a vertex, 0xF empty),
// vertex counts/offsets i32 [C + 1], quad counts/offsets i32 [S + 1], scan block
// sums; then per vertex: reference position float4, corner particles i32 [8],
// weights float [8], side code u32, current position float4; per quad: i32 [4]
// and a cut flag u8.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "tlmpm_common.h"
#include "tlmpm_device.h"

DEV long long site_index(const SurfGrid& G, int x, int y, int z)
{
    if (x < 0 || y < 0 || z < 0 || x >= G.sx || y >= G.sy || z >= G.sz) return -1;
    return ((long long)z * G.sy + y) * G.sx + x;
}

DEV void cube_coords(const SurfGrid& G, long long c, int& x, int& y, int& z)
{
    const long long cx = G.sx + 1, cy = G.sy + 1;
    x = (int)(c % cx) - 1;
    y = (int)((c / cx) % cy) - 1;
    z = (int)(c / (cx * cy)) - 1;
}

DEV long long cube_index(const SurfGrid& G, int x, int y, int z)
{
    return ((long long)(z + 1) * (G.sy + 1) + (y + 1)) * (G.sx + 1) + (x + 1);
}

// sorted particle index of a site, or -1
DEV int site_particle(const SurfGrid& G, const SurfMem& M, int x, int y, int z)
{
    const long long s = site_index(G, x, y, z);
    if (s < 0) return -1;
    const unsigned long long k = M.smap[s];
    return k == ~0ull ? -1 : (int)(k & 0xFFFFFFFFull);
}

__global__ void k_surf_fill(unsigned long long* p, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = ~0ull;
}

// site of every particle; the smallest caller index wins a shared site
__global__ void k_surf_sites(SceneK S, SceneD D, SurfGrid G, SurfMem M)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= S.N) return;
    const double q0 = ((double)D.X[p] - G.ox) / G.h, q1 = ((double)D.X[S.N + p] - G.oy) / G.h,
                 q2 = ((double)D.X[2 * S.N + p] - G.oz) / G.h;
    const long long s = site_index(G, (int)floor(q0), (int)floor(q1), (int)floor(q2));
    if (s < 0) return;
    const unsigned long long key = ((unsigned long long)(unsigned)D.perm[p] << 32) | (unsigned long long)p;
    atomicMin(&M.smap[s], key);
}

// corners of a cube: sorted particle (-1 empty) and side code
struct CubeCorners {
    int p[8];
    uint32_t code[8];
};

DEV CubeCorners load_corners(const SurfGrid& G, const SurfMem& M, const SceneD& D, int x, int y, int z)
{
    CubeCorners c;
#pragma unroll
    for (int k = 0; k < 8; k++) {
        c.p[k] = site_particle(G, M, x + (k & 1), y + ((k >> 1) & 1), z + ((k >> 2) & 1));
        c.code[k] = c.p[k] >= 0 ? (D.code[c.p[k]] & TL_CODE_MASK) : 0u;
    }
    return c;
}

DEV bool cube_intact(const CubeCorners& c, int a, int b)
{
    return c.p[a] >= 0 && c.p[b] >= 0 && !codes_conflict(c.code[a], c.code[b]);
}

// region root of every corner (union by the smaller corner index), -1 when empty
DEV void cube_regions(const CubeCorners& c, int root[8])
{
#pragma unroll
    for (int k = 0; k < 8; k++) root[k] = c.p[k] >= 0 ? k : -1;
    // the 12 edges, in increasing (lower, upper) corner order
    const int ea[12] = {0, 0, 0, 1, 1, 2, 2, 3, 4, 4, 5, 6};
    const int eb[12] = {1, 2, 4, 3, 5, 3, 6, 7, 5, 6, 7, 7};
    for (int e = 0; e < 12; e++) {
        const int a = ea[e], b = eb[e];
        if (!cube_intact(c, a, b)) continue;
        int ra = a, rb = b;
        while (root[ra] != ra) ra = root[ra];
        while (root[rb] != rb) rb = root[rb];
        if (ra != rb) root[max(ra, rb)] = min(ra, rb);
    }
#pragma unroll
    for (int k = 0; k < 8; k++)
        if (root[k] >= 0) {
            int r = k;
            while (root[r] != r) r = root[r];
            root[k] = r;
        }
}

// corner k of the cube has a transition edge (an edge to an empty or conflicting corner)
DEV bool corner_transition(const CubeCorners& c, int k)
{
    return c.p[k] >= 0 && (!cube_intact(c, k, k ^ 1) || !cube_intact(c, k, k ^ 2) || !cube_intact(c, k, k ^ 4));
}

// per cube: regions, the number of vertices and the corner -> vertex map
__global__ void k_surf_cubes(SceneK S, SceneD D, SurfGrid G, SurfMem M)
{
    const long long ci = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (ci >= G.C) return;
    int x, y, z;
    cube_coords(G, ci, x, y, z);
    const CubeCorners c = load_corners(G, M, D, x, y, z);
    int root[8];
    cube_regions(c, root);
    bool has[8] = {false, false, false, false, false, false, false, false}; // region root has a transition
#pragma unroll
    for (int k = 0; k < 8; k++)
        if (corner_transition(c, k)) has[root[k]] = true;
    int idx[8], nv = 0;
#pragma unroll
    for (int k = 0; k < 8; k++) idx[k] = (root[k] == k && has[k]) ? nv++ : -1;
    uint32_t map = 0;
#pragma unroll
    for (int k = 0; k < 8; k++) {
        const uint32_t v = root[k] < 0 ? 0xFu : (idx[root[k]] >= 0 ? (uint32_t)idx[root[k]] : 0xEu);
        map |= v << (4 * k);
    }
    M.creg[ci] = map;
    M.voff[ci] = nv;
}

// directed transitions of a site, in the order d = x, y, z; + then -
DEV int site_transitions(const SurfGrid& G, const SurfMem& M, const SceneD& D, int x, int y, int z, int p,
                         bool tr[6], bool cut[6])
{
    const uint32_t cp = D.code[p] & TL_CODE_MASK;
    int n = 0;
#pragma unroll
    for (int d = 0; d < 3; d++)
#pragma unroll
        for (int sgi = 0; sgi < 2; sgi++) {
            const int sg = sgi == 0 ? 1 : -1;
            const int q = site_particle(G, M, x + (d == 0 ? sg : 0), y + (d == 1 ? sg : 0), z + (d == 2 ? sg : 0));
            const bool conf = q >= 0 && codes_conflict(cp, D.code[q] & TL_CODE_MASK);
            tr[2 * d + sgi] = q < 0 || conf;
            cut[2 * d + sgi] = conf;
            n += tr[2 * d + sgi] ? 1 : 0;
        }
    return n;
}

__global__ void k_surf_site_quads(SceneK S, SceneD D, SurfGrid G, SurfMem M)
{
    const long long si = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (si >= G.S) return;
    const int x = (int)(si % G.sx), y = (int)((si / G.sx) % G.sy), z = (int)(si / ((long long)G.sx * G.sy));
    const unsigned long long k = M.smap[si];
    int n = 0;
    if (k != ~0ull) {
        bool tr[6], cut[6];
        n = site_transitions(G, M, D, x, y, z, (int)(k & 0xFFFFFFFFull), tr, cut);
    }
    M.qoff[si] = n;
}

// ---------------------------------------------------------------- exclusive scan
// In place over a[0..n) with the total in a[n]: per block of 1024 entries a local
// scan and its sum, a one-block scan of the sums, then the block offsets added.
#define TL_SSCAN 1024
__global__ __launch_bounds__(256) void k_surf_scan_local(int* a, long long n, int* bsum)
{
    __shared__ int s_w[4];
    const long long base = (long long)blockIdx.x * TL_SSCAN;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    int v[4], loc = 0;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const long long i = base + 4 * t + j;
        v[j] = i < n ? a[i] : 0;
        loc += v[j];
    }
    int incl = loc;
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(incl, o, 64);
        if (lane >= o) incl += u;
    }
    if (lane == 63) s_w[wv] = incl;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wv; w++) before += s_w[w];
    int run = before + incl - loc;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const long long i = base + 4 * t + j;
        if (i < n) a[i] = run;
        run += v[j];
    }
    if (t == 255) bsum[blockIdx.x] = before + incl;
}

__global__ __launch_bounds__(1024) void k_surf_scan_sums(int* bsum, int nb)
{
    __shared__ int s_c[4096];
    __shared__ int s_w[16];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    int carry = 0;
    for (int base = 0; base < nb; base += 4096) {
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int i = base + k * 1024 + t;
            s_c[k * 1024 + t] = i < nb ? bsum[i] : 0;
        }
        __syncthreads();
        int loc = 0;
#pragma unroll
        for (int k = 0; k < 4; k++) loc += s_c[4 * t + k];
        int incl = loc;
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        if (lane == 63) s_w[wv] = incl;
        __syncthreads();
        int before = 0, total = 0;
        for (int w = 0; w < 16; w++) {
            before += w < wv ? s_w[w] : 0;
            total += s_w[w];
        }
        int run = carry + before + incl - loc;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int c = s_c[4 * t + k];
            s_c[4 * t + k] = run;
            run += c;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int i = base + k * 1024 + t;
            if (i < nb) bsum[i] = s_c[k * 1024 + t];
        }
        carry += total;
        __syncthreads();
    }
    if (t == 0) bsum[nb] = carry;
}

__global__ __launch_bounds__(256) void k_surf_scan_add(int* a, long long n, const int* bsum, int nb)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] += bsum[i / TL_SSCAN];
    if (i == 0) a[n] = bsum[nb];
}

// ------------------------------------------------------------ vertices and quads
// site centre coordinate along axis a
DEV double site_centre(const SurfGrid& G, int a, int s) { return (a == 0 ? G.ox : a == 1 ? G.oy : G.oz) + ((double)s + 0.5) * G.h; }

__global__ void k_surf_vertices(SceneK S, SceneD D, SurfGrid G, SurfMem M)
{
    const long long ci = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (ci >= G.C) return;
    const int v0 = M.voff[ci], nv = M.voff[ci + 1] - v0;
    if (nv == 0) return;
    int x, y, z;
    cube_coords(G, ci, x, y, z);
    const CubeCorners c = load_corners(G, M, D, x, y, z);
    const uint32_t map = M.creg[ci];
    const int m[3] = {x, y, z};
    for (int r = 0; r < nv; r++) {
        // transition midpoints of region r: per axis sum and count along that axis,
        // and over all its transitions
        double sa[3] = {0.0, 0.0, 0.0}, sall[3] = {0.0, 0.0, 0.0};
        int na[3] = {0, 0, 0}, nall = 0;
        uint32_t code = 0;
        for (int k = 0; k < 8; k++) {
            if (((map >> (4 * k)) & 0xFu) != (uint32_t)r) continue;
            code |= c.code[k];
            for (int a = 0; a < 3; a++) {
                const int w = k ^ (1 << a);
                if (cube_intact(c, k, w)) continue;
                double mid[3];
                for (int b = 0; b < 3; b++) {
                    const int sk = m[b] + ((k >> b) & 1);
                    mid[b] = b == a ? site_centre(G, b, m[b]) + 0.5 * G.h : site_centre(G, b, sk);
                }
                sa[a] += mid[a];
                na[a]++;
                for (int b = 0; b < 3; b++) sall[b] += mid[b];
                nall++;
            }
        }
        double pos[3], t[3];
        for (int a = 0; a < 3; a++) {
            pos[a] = na[a] > 0 ? sa[a] / na[a] : sall[a] / nall;
            t[a] = (pos[a] - site_centre(G, a, m[a])) / G.h;
        }
        double wsum = 0.0, wk[8];
        for (int k = 0; k < 8; k++) {
            wk[k] = 0.0;
            if (((map >> (4 * k)) & 0xFu) != (uint32_t)r) continue;
            double w = 1.0;
            for (int a = 0; a < 3; a++) w *= ((k >> a) & 1) ? t[a] : 1.0 - t[a];
            wk[k] = w;
            wsum += w;
        }
        const int v = v0 + r;
        M.vX[v] = make_float4((float)pos[0], (float)pos[1], (float)pos[2], 0.0f);
        M.vcode[v] = code;
        for (int k = 0; k < 8; k++) {
            const bool in = ((map >> (4 * k)) & 0xFu) == (uint32_t)r;
            M.vp[(long long)v * 8 + k] = in ? c.p[k] : -1;
            M.vw[(long long)v * 8 + k] = in ? (float)(wk[k] / wsum) : 0.0f;
        }
    }
}

__global__ void k_surf_quads(SceneK S, SceneD D, SurfGrid G, SurfMem M)
{
    const long long si = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (si >= G.S) return;
    const int q0 = M.qoff[si], nq = M.qoff[si + 1] - q0;
    if (nq == 0) return;
    const int s[3] = {(int)(si % G.sx), (int)((si / G.sx) % G.sy), (int)(si / ((long long)G.sx * G.sy))};
    bool tr[6], cut[6];
    site_transitions(G, M, D, s[0], s[1], s[2], (int)(M.smap[si] & 0xFFFFFFFFull), tr, cut);
    int q = q0;
    for (int d = 0; d < 3; d++) {
        const int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
        for (int sgi = 0; sgi < 2; sgi++) {
            if (!tr[2 * d + sgi]) continue;
            const int sg = sgi == 0 ? 1 : -1;
            int ring[4];
            const int o1[4] = {-1, 0, 0, -1}, o2[4] = {-1, -1, 0, 0};
            for (int j = 0; j < 4; j++) {
                int mc[3];
                mc[d] = sg > 0 ? s[d] : s[d] - 1;
                mc[e1] = s[e1] + o1[j];
                mc[e2] = s[e2] + o2[j];
                const long long ci = cube_index(G, mc[0], mc[1], mc[2]);
                const int k = (s[0] - mc[0]) | ((s[1] - mc[1]) << 1) | ((s[2] - mc[2]) << 2);
                const uint32_t r = (M.creg[ci] >> (4 * k)) & 0xFu;
                ring[j] = M.voff[ci] + (int)r;
            }
            M.quads[q] = sg > 0 ? make_int4(ring[0], ring[1], ring[2], ring[3])
                                : make_int4(ring[3], ring[2], ring[1], ring[0]);
            M.qcut[q] = cut[2 * d + sgi] ? 1 : 0;
            q++;
        }
    }
}

// current vertex positions: reference position plus the weighted displacement of
// the region's particles
__global__ void k_surf_embed(SceneK S, SceneD D, SurfMem M, int nv)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const float4 X = M.vX[v];
    float d[3] = {0.0f, 0.0f, 0.0f};
    for (int k = 0; k < 8; k++) {
        const int p = M.vp[(long long)v * 8 + k];
        if (p < 0) continue;
        const float w = M.vw[(long long)v * 8 + k];
        d[0] += w * D.u[p];
        d[1] += w * D.u[S.N + p];
        d[2] += w * D.u[2 * S.N + p];
    }
    M.vx[v] = make_float4(X.x + d[0], X.y + d[1], X.z + d[2], 0.0f);
}

static unsigned grid_of(long long n, int t) { return (unsigned)((n + t - 1) / t); }

static hipError_t scan(int* a, long long n, int* bsum, hipStream_t st)
{
    const int nb = (int)((n + TL_SSCAN - 1) / TL_SSCAN);
    hipLaunchKernelGGL(k_surf_scan_local, dim3(nb), dim3(256), 0, st, a, n, bsum);
    hipLaunchKernelGGL(k_surf_scan_sums, dim3(1), dim3(1024), 0, st, bsum, nb);
    hipLaunchKernelGGL(k_surf_scan_add, dim3(grid_of(n + 1, 256)), dim3(256), 0, st, a, n, bsum, nb);
    return hipGetLastError();
}

extern "C" {
// topology counts: site table, cube regions, vertex and quad offsets (totals at
// voff[C] and qoff[S])
hipError_t tl_surface_count(const SceneK* S, const SceneD* D, const SurfGrid* G, const SurfMem* M, hipStream_t st)
{
    hipLaunchKernelGGL(k_surf_fill, dim3(grid_of(G->S, 256)), dim3(256), 0, st, M->smap, G->S);
    if (S->N > 0) hipLaunchKernelGGL(k_surf_sites, dim3(grid_of(S->N, 256)), dim3(256), 0, st, *S, *D, *G, *M);
    hipLaunchKernelGGL(k_surf_cubes, dim3(grid_of(G->C, 256)), dim3(256), 0, st, *S, *D, *G, *M);
    hipLaunchKernelGGL(k_surf_site_quads, dim3(grid_of(G->S, 256)), dim3(256), 0, st, *S, *D, *G, *M);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan(M->voff, G->C, M->bsum, st);
    if (e != hipSuccess) return e;
    return scan(M->qoff, G->S, M->bsum, st);
}

hipError_t tl_surface_fill(const SceneK* S, const SceneD* D, const SurfGrid* G, const SurfMem* M, hipStream_t st)
{
    hipLaunchKernelGGL(k_surf_vertices, dim3(grid_of(G->C, 256)), dim3(256), 0, st, *S, *D, *G, *M);
    hipLaunchKernelGGL(k_surf_quads, dim3(grid_of(G->S, 256)), dim3(256), 0, st, *S, *D, *G, *M);
    return hipGetLastError();
}

hipError_t tl_surface_embed(const SceneK* S, const SceneD* D, const SurfMem* M, int nv, hipStream_t st)
{
    if (nv > 0) hipLaunchKernelGGL(k_surf_embed, dim3(grid_of(nv, 256)), dim3(256), 0, st, *S, *D, *M, nv);
    return hipGetLastError();
}
}
