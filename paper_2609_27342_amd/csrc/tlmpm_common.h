// tlmpm_common.h -- structures shared by the host runtime and the gfx950 kernels.
//
// Layout in HBM (one scene, all carved from the caller's workspace):
//   particles, sorted by (brick, cell parity class, cell, input order), SoA float:
//     X[3][N] reference positions, u[3][N] = x - X, v[3][N], H[9][N] = F - I
//   code[N]      u32: side mask s1 (bits 0-14: digit == 1), s2 (bits 15-29: digit == 2),
//                bit 30: code_prev[p] holds the code the pending F update must use,
//                bit 31: material-contact candidate
//   grid: node ids are brick-major, id = nodebrick * 64 + (lz * 16 + ly * 4 + lx)
//     slot tables (two buffers): count[node] u8, code[S_CAP][node] u32 (ascending)
//     P2G partials  [8 contributors][S_CAP][node][8] float  (m, p, dp, pad)
//     MUSL partials [8 contributors][S_CAP][node][4] float  (m, p~)
#pragma once
#include <stdint.h>

#define TL_B 4                 // cells per brick edge
#define TL_CELLS 64            // cells per brick
#define TL_BOXN 125            // nodes of a brick's (TL_B + 1)^3 box
#define TL_SCAP_MAX 16         // largest per-node capacity of logical grids (slots)
#define TL_BOX_SLOTS 640       // slots of one brick box held in LDS
#define TL_MAX_TOOLS 4          // tools per scene (rigid-history slots 1..4; slot 0 = floor)
#define TL_WG 512              // threads per brick workgroup: 8 waves = 8 parity classes
#define TL_STATIC_SCRATCH_BYTES (16u << 20) // workspace of a batch that allocates nothing (16 MiB)
#define TL_STATIC_DEVICES 8    // GPUs of one process that can hold such a batch
#define TL_STATIC_MAX_SCENES 1024 // scenes of such a batch (its host staging is static)

#define TL_CODE_MASK 0x3FFFFFFFu
#define TL_PREV_BIT 0x40000000u
#define TL_CAND_BIT 0x80000000u

// status bits (device, sticky)
#define TL_ST_NONFINITE 1
#define TL_ST_SLOT 2
#define TL_ST_BOX 4
#define TL_ST_LOOKUP 8
#define TL_ST_CONTACT 16

#define TL_CC_EMPTY 0xFFFFFFFEu // cell summary: no particle
#define TL_CC_MIXED 0xFFFFFFFFu // cell summary: more than TL_CKEYS slot keys (scan the particles)
#define TL_CC_FEW 0xC0000000u   // cell summary: TL_CC_FEW | n, 2 <= n <= TL_CKEYS keys listed in ckeys
#define TL_CKEYS 4
#define TL_GMAX 8              // same-code groups (of <= 8 particles) per cell in a mixed brick
#define TL_PCAP 16             // persistent pair springs kept per particle (all its partners)
#define TL_HSLOTS 64  // slots of the speed-bound maximum (spreads the atomics)
#define TL_HSTRIDE 1  // ints between slots (consecutive: cheap to read in every binning block)
#define TL_USLOTS 64  // slots of each displacement bound
#ifndef TL_PLANES
#define TL_PLANES 4            // lanes per candidate in the pair search (4 or 8)
#endif
#define TL_PCAND (256 / TL_PLANES) // candidates per pair-search block (256 threads)
#define TL_BCAP 8              // candidate records stored inline per hash bucket

// tool flags (same values as the ABI)
#define TL_TOOL_LABELS 1u
#define TL_TOOL_CONTACT 2u
#define TL_TOOL_CUTTING 4u
#define TL_TOOL_ADVANCE 8u

struct DevBlade {
    double xe[3], n[3], e[3], d[3], ve[3];
    double half_len, half_width, b_back, b_lead;
    int cut, new_cut;
};

// A tool as the kernels see it (device memory).  With TL_TOOL_ADVANCE the pose of
// substep j is the stored pose translated by (j dt) times the velocity.
struct DevTool {
    DevBlade b;
    double xB[3], vB[3];
    float wB[3];
    float invm;    // constant part of the inverse effective mass
    float imass;   // 1/M of a free tool
    float iinv[9]; // world-frame inverse inertia about xB
    unsigned flags;
    int slot; // rigid-history slot 1..TL_MAX_TOOLS (0 is the floor)
};

// scalar parameters of a scene, passed to every kernel by value
struct SceneK {
    long long N;
    int cx, cy, cz;       // cells
    int cbx, cby, cbz;    // cell bricks
    int nbx, nby, nbz;    // node bricks
    long long NN;         // node ids = nbx*nby*nbz*64
    double ox, oy, oz, dx, inv_dx_d;
    float inv_dx;
    float dt, beta, gx, gy, gz;
    float nu;
    int e_uniform, m_uniform, v_uniform;
    float E0, m0, V0;
    float s_R, s_n, gamma_k, gamma_c, mu_s, mu_d;
    float Rmax;           // largest contact radius s_R V0^{1/3} / 2
    int floor_on;
    float floor_z;
    float G_c, zeta, u_min;
    int single_field;
    int material_contact;
    int scap;         // slot capacity per node (<= TL_SCAP_MAX)
    int material;     // 0 Neo-Hookean, 1 fixed-corotated
    float visc;       // Newtonian viscosity
    float ystress;    // von Mises yield stress (0: elastic)
    int pair_blocks;  // blocks of the pair search (grid-stride over the candidates)
    int stencil;      // 0 trilinear (8 nodes), 1 quadratic B-spline (27 nodes)
    int xcap;         // workgroups for the later rounds of mixed bricks (used while xlist fits)
    int pair_skip;    // the binning may mark candidates that provably have no contact partner
                      // (material contact, trilinear stencil: its G2P keeps the displacement anchors)
    double dt_d;
};

// device pointers of a scene
struct SceneD {
    float* X;      // [3][N]
    float* u;      // [3][N]
    float* v;      // [3][N]
    float* H;      // [9][N]
    uint32_t* code;
    uint32_t* code_prev;
    float* D;
    int* perm;     // sorted index -> caller's index
    float* E;      // [N] or null
    float* m;      // [N] or null
    float* V0;     // [N] or null
    int* cell_start;   // [n_bricks*64 + 1]
    int* active;       // active brick ids
    int n_active;
    uint8_t* cnt[2];
    uint32_t* scode[2];
    float* p2g;    // [active brick][scap][125 box nodes][8]: each brick's P2G box sums
    float* rs;     // [active brick][scap][125 box nodes][4]: each brick's re-scatter box sums
    float* p2g_x;  // the same two for the later same-code rounds of a split brick
    float* rs_x;
    int* xp2g;     // [active brick] p2g_x holds this substep's sums of the brick (split)
    int* xrs;      // [active brick] rs_x (and aabb_x) hold the brick's last G2P sums (split)
    float* aabb_x; // [n_bricks][8] box of a split brick's later rounds
    int* xlist;    // [active brick] active indices of the bricks with a mixed cell (count: ctr[3])
    int* xin;      // [active brick] the brick is in xlist
    int* xg;       // [1] the last G2P split the mixed bricks (rs_x, xrs, aabb_x in use)
    int* bact;     // [bricks] active index of a brick, -1 if it holds no particle
    float* hist;   // rigid contact history [TL_MAX_TOOLS+1][4][N]: u_t xyz, stamp
    float* aabb;   // [n_bricks][8]: min xyz, max xyz, max |v|, 0
    double* wpart; // [TL_MAX_TOOLS * 6][n_active] per-brick wrench sums of the call so far
    float* Fdot;   // [9][N] rate of F of its last update (viscous scenes), else null
    float* Gp;     // [9][N] F_p^{-1} - I (plastic scenes), else null
    double* wacc;  // [TL_MAX_TOOLS][6]
    float* Jmat;   // [3][N] material contact impulse (candidates only)
    float* Jrig;   // [3][N] floor and tool impulse (bricks with brig set)
    int* brig;     // [bricks] the brick was within reach of a rigid body this substep
    int* bmixed;   // [bricks] a cell of the brick holds two side codes
    uint32_t* ccode; // [bricks * 64] (sorted cell order) the one slot key of a cell, or TL_CC_*
    uint32_t* ckeys; // [bricks * 64][TL_CKEYS] ascending keys of a cell summarised as TL_CC_FEW
    int* gmeta;      // [active bricks][64 cells][TL_GMAX] groups of a mixed brick: offset << 4 | count
    int* gperm;      // [N] particles of mixed bricks in group order, over each cell's range
    int* bround;     // [active bricks] rounds (largest group count of a cell) of a mixed brick
    DevTool* tools;   // [TL_MAX_TOOLS] tools (or label-only blades) of the current call
    int* tinfo;       // [4] per call: number of tools, any tool with contact, new cut, unused
    int* ctr;         // [4] persistent: contact-history stamp, F update pending, substep of the
                      // call, number of bricks in xlist
    int* status;
    int* dirty;
    int* bdirty;        // [bricks] side codes of the brick changed in the last label pass
    int* pcell;         // [N] cell slot (sorted cell order) of every particle
    // material contact
    uint32_t* cmask;    // [cells] OR of the codes of each cell (sorted cell order)
    uint8_t* cstatic;   // [cells] cell has an empty or out-of-grid neighbour
    int* bcand;         // [active bricks] number of candidates of the brick
    int* cand_idx;      // [N] candidates of each brick, stored over the brick's particle range
    int* coff;          // [active bricks + 1] first global candidate index of each active brick
    float* hbin;        // bin edge (device scalar)
    int* hmax;          // [TL_HSLOTS] largest brick speed bounds for the next binning (float bits)
    float* uanc;        // [bricks][4] displacement anchor a (3) and spread s of the brick's particles,
                        // |u_p - a|_inf <= s after the last G2P (pair-search skip)
    float* uanc_x;      // [bricks][4] the same for the later rounds of a split brick
    float* uref;        // [bricks][4] centre of the box of the brick's reference positions (static)
    uint32_t* bor;      // [bricks] OR of the side keys of the brick's particles
    uint32_t* umm;      // [6][TL_USLOTS] scene bounds of the anchors of the bricks with candidates:
                        // a + s per axis, then s - a (ordered float keys, maximum over the slots;
                        // cleared by the pair pass)
    uint32_t hmask;     // buckets - 1 (power of two)
    int* bcount;        // [2][buckets] entries of each bucket (buffer = stamp parity; the
                        // pair pass clears the other buffer for the next substep)
    int* bids;          // [buckets][TL_BCAP] global candidate indices in arrival order
    float4* crec;       // [N][3] record of each global candidate (dense, brick by brick)
    unsigned long long* htab; // [buckets] overflow lists: generation << 32 | head
    int* hnext;         // [N] overflow list links (global candidate indices)
    int* ph_n;          // [2][N] stamp << 8 | count of owned springs
    int* ph_q;          // [2][N][TL_PCAP] partner of each spring
    float* ph_u;        // [2][N][TL_PCAP][3] spring, oriented for the pair's lower index
    // quadratic stencil
    uint32_t* qcode;    // [2][scap][NN] side keys of the node slots by substep parity (~0u: free)
    float* qacc;        // [NN][scap][8] P2G sums m, p, dp; after the grid update m, v^n, dv
    float* qrs;         // [NN][scap][4] re-scatter sums of m v^{n+1}; after the remap v~
    int* qnodes;        // nodes of the 7x7x7 boxes of the active bricks (ascending)
    int n_qnodes;
    int* qround;        // [active bricks + 1] first lane-map round of each brick
    int* qmap;          // [rounds][512] particle of thread h * 64 + l: cell slot l, half pattern h (-1: none)
};

// Surface reconstruction (tlmpm_surface.hip): the site lattice of one scene and
// the arrays of a surface workspace
struct SurfGrid {
    int sx, sy, sz;       // sites per axis (2 x cells)
    long long S, C;       // sites, cubes ((sx + 1)(sy + 1)(sz + 1), min corner -1 .. s - 1)
    double ox, oy, oz, h; // origin, site spacing
};

struct SurfMem {
    unsigned long long* smap;
    uint32_t* creg;
    int* voff; // [C + 1]: counts, then exclusive offsets
    int* qoff; // [S + 1]
    int* bsum; // scan block sums
    float4* vX;
    int* vp;     // [nv][8]
    float* vw;   // [nv][8]
    uint32_t* vcode;
    float4* vx;
    int4* quads;
    uint8_t* qcut;
};


// Workgroups are dealt to the 8 XCDs (each with its own L2) round-robin by
// dispatch index.  xcd_order(b, G) maps dispatch index b of G to a work index such
// that the workgroups of one XCD take one contiguous range of work items, so
// neighbouring items share an L2.  Used by the batched P2G / G2P launches, whose
// many small scenes fit the L2s (measured faster there; slower for one large
// scene, which keeps the dispatch order).
__device__ __forceinline__ int xcd_order(int b, int G)
{
    const int r = b & 7, q = G >> 3, extra = G & 7;
    return r * q + (r < extra ? r : extra) + (b >> 3);
}

// Value of lane (lane ^ M), M in {1, 2, 4}, by DPP row moves (no LDS traffic):
// quad permutations for 1 and 2; for 4, lanes with bit 2 clear read lane + 4
// (row shift left) and the others lane - 4 (row shift right), all within a row of
// 16 lanes.
template <int M>
__device__ __forceinline__ float lane_xor(float v)
{
    const int x = __float_as_int(v);
    if constexpr (M == 1) {
        return __int_as_float(__builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, true));
    } else if constexpr (M == 2) {
        return __int_as_float(__builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, true));
    } else {
        static_assert(M == 4, "lane_xor: 1, 2 or 4");
        const int up = __builtin_amdgcn_mov_dpp(x, 0x104, 0xF, 0xF, true);
        const int dn = __builtin_amdgcn_mov_dpp(x, 0x114, 0xF, 0xF, true);
        return __int_as_float((threadIdx.x & 4) ? dn : up);
    }
}

// Launch context: one scene (parameters by value) or a batch of scenes (device
// arrays of SceneK / SceneD and, per kind of work item, a list of (scene, block)).
enum { IT_BRICK = 0, IT_NODE, IT_CELL, IT_WRENCH, IT_SCENE, IT_PART, IT_BFLAG, IT_PAIR, IT_XBRICK, TL_ITEM_KINDS };

struct TlLaunch {
    const SceneK* S;   // single scene (host copies), or null in batch mode
    const SceneD* D;
    const SceneK* Ks;  // batch mode: device arrays
    const SceneD* Ds;
    const int2* items[TL_ITEM_KINDS];
    int n_items[TL_ITEM_KINDS];
    int any_material;  // some scene has material contact
    int general;       // some scene needs the general constitutive path (fixed-corotated,
                       // viscosity or plasticity)
    hipStream_t st;
};
