/*
 * tlmpm.h -- C ABI of the MI355X (gfx950) TLMPM cutting library.
 *
 * One substep of total-Lagrangian MPM with persistent ternary side labels, as in
 * BladeMaster (arXiv 2609.27342):
 *   - online side-label assignment from the swept blade (Sec. III-C, Eqs. 3, 4, 6, 7);
 *   - tool-material contact with directional contact work (Sec. III-E, Eqs. 5, 14-16)
 *     and material-material contact (Eqs. 10-13);
 *   - label-masked P2G of mass, momentum and internal force on the fixed reference
 *     grid (Sec. III-B, Eqs. 1, 2);
 *   - compatibility coupling and the grid update (Sec. III-D, Eqs. 8, 9);
 *   - PIC/FLIP G2P of v and x, MUSL re-scatter with the same coupling and the
 *     deformation-gradient update (Sec. III-B, App. Eq. 17).
 * Per scene: Neo-Hookean or fixed-corotated elasticity with Newtonian viscosity and
 * von Mises plasticity (Sec. III-B), trilinear or quadratic B-spline interpolation
 * (Eq. 1), prescribed or free (two-way coupled) tools (Sec. III-A, III-E, III-G).
 *
 * Conventions
 *   - Every call returns a tlmpm_status; nothing throws across the ABI.  The text of
 *     the last error of the calling thread is returned by tlmpm_last_error().
 *   - Host arrays are owned by the caller and only read during the call.
 *   - Device memory: the caller provides ONE device workspace of at least
 *     tlmpm_scene_footprint() bytes (for instance a torch uint8 tensor) and keeps it
 *     alive until tlmpm_destroy_scene().  The library never allocates device memory.
 *   - Streams: the caller's HIP stream (hipStream_t passed as void*; NULL = default).
 *     Calls are asynchronous on that stream except tlmpm_read_state, tlmpm_write_state,
 *     tlmpm_get_status and a tlmpm_step given a non-NULL wrench pointer, which
 *     synchronise it.
 *   - Device-side failures (non-finite state, det F <= 0, too many logical grids at a
 *     node) are sticky per scene and reported by the next synchronising call.
 *   - A scene is used by one host thread at a time.
 */
#ifndef TLMPM_H
#define TLMPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TLMPM_OK = 0,
    TLMPM_E_INVALID = 1,       /* bad argument, particle outside the grid, bad blade frame */
    TLMPM_E_NOMEM = 2,         /* workspace smaller than tlmpm_scene_footprint() */
    TLMPM_E_DEVICE = 3,        /* a HIP runtime call failed */
    TLMPM_E_SLOT_OVERFLOW = 4, /* more logical grids at a node than slot_capacity */
    TLMPM_E_NONFINITE = 5      /* non-finite state or det F <= 0 */
} tlmpm_status;

typedef struct tlmpm_scene tlmpm_scene; /* opaque */

/* Scene description (SI units).  Host arrays are array-of-structs as given. */
typedef struct {
    int64_t n;              /* number of particles (material points) */
    const float* X;         /* [n][3] reference positions X_p (Sec. III-A) */
    const float* v0;        /* [n][3] initial velocities, or NULL for zero; F0 = I */
    const float* vol0;      /* [n] reference volumes V_p^0, or NULL => vol0_uniform */
    const float* mass;      /* [n] masses m_p, or NULL => mass_uniform */
    const float* E;         /* [n] Young's moduli, or NULL => E_uniform */
    float vol0_uniform, mass_uniform, E_uniform;
    float nu;               /* Poisson ratio */
    double dx;              /* reference grid spacing */
    double origin[3];       /* position of reference node (0,0,0) */
    int32_t cells[3];       /* reference cells per axis; every X must lie inside */
    double dt;              /* substep size */
    float gravity[3];
    float flip_beta;        /* PIC/FLIP blend of Eq. 17 */
    /* contact (Sec. III-E): radius scale, normal scale, tangential stiffness and
     * damping scales, static and dynamic friction */
    float s_R, s_n, gamma_k, gamma_c, mu_s, mu_d;
    int32_t material_contact;  /* material-material contact on */
    int32_t floor_on;          /* rigid half-space z >= floor_z, outward normal +z */
    float floor_z;
    float G_c, zeta, u_min;    /* cutting-work threshold parameters (Eq. 5) */
    int32_t max_cuts;          /* K, number of ternary digits (1..15) */
    int32_t single_field;      /* 1: ignore codes (one logical grid), a negative control */
    int32_t slot_capacity;     /* logical grids per node (compact slots, Sec. III-G), 1..16; 0 = 8.
                                  More distinct codes at a node set TLMPM_E_SLOT_OVERFLOW. */
    int32_t material;          /* constitutive model (Sec. III-B): 0 compressible Neo-Hookean,
                                  1 fixed-corotated, P = 2 mu (F - R) + lambda (J - 1) J F^-T */
    float viscosity;           /* Newtonian viscosity eta >= 0 (Pa s): adds J eta (l + l^T) F^-T,
                                  l = dF/dt F^-1 from the last deformation-gradient update */
    float yield_stress;        /* von Mises yield stress (Pa) of the plasticity projection with
                                  material 1; 0 = elastic */
    int32_t stencil;           /* interpolation of Eq. 1: 0 trilinear hat over the base cell's 8
                                  corners, 1 quadratic B-spline over 27 nodes (base node
                                  floor(q - 1/2), q = (X - origin)/dx).  The quadratic stencil
                                  needs every particle at least half a cell inside the grid and
                                  runs one scene per call (batches refuse it); its sums use
                                  floating-point atomics (not bitwise reproducible). */
} tlmpm_scene_desc;

/* A blade record: the cut frame of Eq. 3 and the band of Eq. 4.  (n, e, d) must be
 * orthonormal with d pointing toward the cutting front.  Doubles: the side
 * predicates are evaluated in FP64. */
typedef struct {
    int32_t cut_index;       /* k: the ternary digit this blade assigns, 0..max_cuts-1 */
    int32_t new_cut;         /* nonzero: start of cut k, reset D_p := 0 (Sec. III-A) */
    double x_e[3];           /* point at the middle of the blade edge */
    double n[3], e[3], d[3]; /* plane normal, edge axis, front direction */
    double v_e[3];           /* velocity of x_e */
    double half_len;         /* L_k: half length of the edge */
    double half_width;       /* h_k: band half width (the paper uses 6 dx) */
    double b_back;           /* band rear extent; also the blade height behind the edge */
    double b_lead;           /* band lead extent */
} tlmpm_blade;

#define TLMPM_TOOL_LABELS 1u   /* assign side digits from the blade band each substep */
#define TLMPM_TOOL_CONTACT 2u  /* tool-material contact (Eqs. 14-16) */
#define TLMPM_TOOL_CUTTING 4u  /* directional contact work and release (Eq. 5) */
#define TLMPM_TOOL_ADVANCE 8u  /* translate the pose by dt * velocity after each substep */

/* A rigid tool: the zero-thickness rectangle of its blade record, |l| <= half_len
 * along e and -b_back <= f <= 0 along d, in the plane s = 0, moving with the twist
 * (v_B, omega_B) about x_B.  Its inverse effective mass at a contact point x_c
 * along the contact normal n (Sec. III-E, Eq. 15) is
 *   w = w_B + inv_mass + (r x n) . inv_inertia (r x n),  r = x_c - x_B,
 * so a kinematically prescribed tool has all three zero, and a free rigid body
 * has x_B at its centre of mass, inv_mass = 1/M and inv_inertia = I^-1 in world
 * axes (tlmpm_rigid_tool fills these from a tlmpm_rigid_body). */
typedef struct {
    tlmpm_blade blade;
    double x_B[3];     /* torque reference point of the tool (Eq. 16); centre of mass */
    double v_B[3];     /* linear velocity */
    double omega_B[3]; /* angular velocity */
    double w_B;        /* constant part of the inverse effective mass */
    uint32_t flags;    /* TLMPM_TOOL_* */
    int32_t reserved;
    double inv_mass;       /* 1/M of a free tool, else 0 */
    double inv_inertia[9]; /* world-frame inverse inertia about x_B, row major, else 0 */
} tlmpm_tool;

/* Device bytes a scene of this description needs (depends on n, cells and the
 * contact switches only). */
tlmpm_status tlmpm_scene_footprint(const tlmpm_scene_desc* desc, size_t* device_bytes);

/* Build a scene: validates the description, sorts particles by reference cell,
 * carves the caller's workspace and uploads the state on `hip_stream`. */
tlmpm_status tlmpm_create_scene(const tlmpm_scene_desc* desc, void* dev_workspace, size_t bytes,
                                void* hip_stream, tlmpm_scene** out);

tlmpm_status tlmpm_destroy_scene(tlmpm_scene* scene);

/* ---- Two-way tool coupling (Sec. III-A, III-E, III-G).  The paper leaves the
 * tool's rigid-body dynamics to an external solver that receives the interval-
 * averaged wrench of tlmpm_step and returns the next pose and twist; these two
 * host-only calls are such a solver for a free rigid tool (a knife released under
 * gravity): tlmpm_rigid_step advances the body, tlmpm_rigid_tool turns it into the
 * tool record of the next interval (pose and twist held over the interval). */
typedef struct {
    double x[3];       /* centre of mass, world */
    double q[4];       /* orientation, unit quaternion (w, x, y, z), body -> world */
    double v[3];       /* velocity of the centre of mass */
    double omega[3];   /* angular velocity, world axes */
    double mass;       /* M > 0 */
    double inertia[3]; /* principal moments of inertia about the centre of mass (body axes) */
} tlmpm_rigid_body;

/* One step of length h > 0 of the Newton-Euler equations under the wrench
 * [6] = (force, torque about x) and gravity, semi-implicit (symplectic) Euler:
 *   v += h (F / M + g);  omega_b += h I^-1 (tau_b - omega_b x I omega_b) in body axes;
 *   x += h v;  q += (h / 2) (0, omega) q, renormalised.
 * TLMPM_E_INVALID for a null pointer, h <= 0, M or a moment <= 0, a zero or
 * non-finite quaternion, or a non-finite result (the body is then unchanged). */
tlmpm_status tlmpm_rigid_step(tlmpm_rigid_body* body, const double wrench[6], const double gravity[3], double h);

/* Tool record of a blade fixed to the body: blade_body holds x_e, n, e, d in body
 * axes relative to the centre of mass (its v_e is ignored) and the band sizes, cut
 * index and new-cut flag, which are copied.  Output in world axes: x_e = x + R x_e,
 * n, e, d rotated, v_e = v + omega x (x_e - x); x_B = x, v_B = v, omega_B = omega,
 * w_B = 0, inv_mass = 1/M, inv_inertia = R diag(1/I) R^T; flags as given.
 * TLMPM_E_INVALID for null pointers or a body that tlmpm_rigid_step would refuse. */
tlmpm_status tlmpm_rigid_tool(const tlmpm_rigid_body* body, const tlmpm_blade* blade_body, uint32_t flags,
                              tlmpm_tool* out);

/* Side-label pass (Eqs. 3, 4, 6) on the stored x^n, v^n for each blade in turn.
 * Digits only go 0 -> 1 or 2.  A blade with new_cut first resets D to zero for
 * every particle.  Labels govern the next substep's contact and P2G. */
tlmpm_status tlmpm_assign_labels(tlmpm_scene* scene, const tlmpm_blade* blades, int32_t n_blades);

/* n_substeps TLMPM substeps.  Each substep: label pass for tools with
 * TLMPM_TOOL_LABELS, contact, P2G, coupling, grid update, G2P, re-scatter; the
 * deformation-gradient update of a substep is completed lazily by the next one
 * (or by tlmpm_read_state; with the quadratic stencil within the substep).  The tool pose is held fixed over the substeps unless
 * TLMPM_TOOL_ADVANCE is set.  wrench: NULL, or [n_tools][6] (force, torque on each
 * tool) averaged over the substeps so that it carries the same impulse (Sec.
 * III-G); a non-NULL pointer synchronises. */
tlmpm_status tlmpm_step(tlmpm_scene* scene, const tlmpm_tool* tools, int32_t n_tools, int32_t n_substeps,
                        double* wrench);

#define TLMPM_FIELD_X 1u      /* float [n][3] reference positions */
#define TLMPM_FIELD_U 2u      /* float [n][3] displacement x - X */
#define TLMPM_FIELD_V 4u      /* float [n][3] velocity */
#define TLMPM_FIELD_F 8u      /* float [n][9] deformation gradient, row major */
#define TLMPM_FIELD_CODE 16u  /* uint64 [n] ternary code sum_k d_k 3^k (Eq. 7) */
#define TLMPM_FIELD_D 32u     /* float [n] cutting progress */
#define TLMPM_FIELD_DIGITS 64u /* uint8 [n][max_cuts] ternary digits */
#define TLMPM_FIELD_H 128u     /* float [n][9] H = F - I, row major: the stored form of F, which
                                  keeps small strains to FP32 relative precision (F in FP32
                                  rounds them to multiples of 2^-24) */

/* Copy fields to host buffers in the caller's original particle order.  host_out
 * has one pointer per bit of field_mask, in increasing bit order.  Synchronises. */
tlmpm_status tlmpm_read_state(tlmpm_scene* scene, uint32_t field_mask, void* const* host_out);

/* Overwrite fields from host buffers (original order; same layout as read_state;
 * TLMPM_FIELD_X and TLMPM_FIELD_CODE are not writable; F and H not both in one call).  For restarts and
 * shared-input comparisons.  Synchronises. */
tlmpm_status tlmpm_write_state(tlmpm_scene* scene, uint32_t field_mask, const void* const* host_in);

/* Sticky device status of the scene (a tlmpm_status value, 0 = OK).  Synchronises. */
tlmpm_status tlmpm_get_status(tlmpm_scene* scene, int32_t* status);

/* Diagnostics: number of occupied logical-grid slots over all nodes and the
 * largest count at one node (Sec. III-G, compact slots).  Synchronises. */
tlmpm_status tlmpm_slot_stats(tlmpm_scene* scene, int64_t* total_slots, int32_t* max_per_node);

/* Diagnostics: hist[c] = number of grid nodes holding c logical-grid slots,
 * c = 0..16 (Sec. III-G, compact slots; Fig. 10b counts the occupied slots).
 * Synchronises. */
tlmpm_status tlmpm_slot_histogram(tlmpm_scene* scene, int64_t hist[17]);

/* Diagnostics of the material-contact search of the last substep (Sec. III-E):
 * out[0] contact candidates, out[1] hash buckets, out[2] occupied buckets,
 * out[3] buckets holding more candidates than their inline records, out[4] the
 * largest bucket count, out[5] the bin edge in metres, out[6] the pairs in contact
 * (each contact is kept by both partners, at most 16 per particle; half the sum of
 * the particles' counts), out[7] the candidates whose search the binning skipped
 * (no partner possible: every particle within the bin edge is a reference neighbour
 * with a compatible code).  All zero without material contact.  Synchronises. */
tlmpm_status tlmpm_contact_stats(tlmpm_scene* scene, double out[8]);

/* Launch-shape settings, process-wide.  A scene takes them when it is created
 * (and tlmpm_batch_scene_bytes reads them), so set them before creating the scenes
 * they are meant for; scenes created earlier keep theirs.  They change how work is
 * divided among workgroups, not what is computed: the pair search and the stream
 * arrangement give bitwise the same results for any setting; splitting mixed bricks
 * adds a brick's later same-code rounds as a second partial, which changes the
 * rounding of those sums (a batch equals its scenes run alone when all were
 * created with the same settings).
 *   pair_div, pair_cap: pair-search workgroups of a scene = min(pair_cap,
 *       max(1, N / pair_div)) (defaults 128, 4096);
 *   split_lo, split_hi, split_div, split_cap: scenes of split_lo..split_hi active
 *       bricks run the later rounds of bricks with a mixed cell in min(split_cap,
 *       active / split_div) extra workgroups of P2G and G2P (512, 4096, 4, 256;
 *       split_cap 0 turns the split off);
 *   one_stream_bricks: a single scene of at most this many active bricks runs a
 *       substep with a label pass on one stream (label pass and rigid contact in
 *       one launch, slot tables and pair search in one launch), larger ones put
 *       rigid contact and the slot tables on a second stream (2048);
 *   pair_skip: 1 lets the binning mark the material-contact candidates that
 *       provably have no partner, whose search the pair pass then skips (Sec.
 *       III-E; bitwise the same results), 0 searches every candidate (1).
 * tlmpm_set_tuning(NULL) restores the defaults; TLMPM_E_INVALID for values out of
 * range (a divisor or cap below 1, split_hi < split_lo, a negative value,
 * pair_skip other than 0 or 1). */
typedef struct {
    int32_t pair_div, pair_cap;
    int32_t split_lo, split_hi, split_div, split_cap;
    int32_t one_stream_bricks;
    int32_t pair_skip;
} tlmpm_tuning;
tlmpm_status tlmpm_set_tuning(const tlmpm_tuning* tuning);
tlmpm_status tlmpm_get_tuning(tlmpm_tuning* tuning);

/* HIP graph replay of substeps.  While enabled, a tlmpm_step of n >= 3 substeps
 * runs its first substep as plain launches and the following pairs of substeps as
 * replays of a captured graph of those launches (one graph per combination of
 * label pass, tool contact and rigid contact, built on first use and kept until
 * the scene is destroyed).  Results are bitwise those of plain launches; every
 * per-substep value the kernels read is in device memory.  Off while kernel timing
 * is on.  Default: off. */
tlmpm_status tlmpm_set_graphs(tlmpm_scene* scene, int32_t enable);

/* Kernel timing (diagnostics).  enable = 1: every kernel the scene launches is
 * bracketed by HIP events on the scene's stream (each kernel then has a launch of
 * its own, on one stream).  enable = 2: only the P2G and G2P launches are
 * bracketed, the launch arrangement is unchanged (for timing those two inside a
 * measured run).  0: off.  tlmpm_profile_read synchronises and returns, per kernel
 * class (0 P2G, 1 grid update + G2P, 2 labels, 3 slot tables, 4 material contact,
 * 5 other), the summed duration in ms and the launch count, then clears the
 * record.  n_classes: length of both output arrays (<= 6). */
tlmpm_status tlmpm_profile_enable(tlmpm_scene* scene, int32_t enable);
tlmpm_status tlmpm_profile_read(tlmpm_scene* scene, int32_t n_classes, double* ms, int64_t* launches);

/* ---- Surface reconstruction for visualisation (Sec. III-F), outside the substep.
 * The surface of the scene's current side codes on the 2x2x2 sub-cell lattice of
 * the reference grid (site spacing dx / 2, site floor((X - origin) / (dx / 2)) per
 * axis; a site is material when a particle lies in it, the one of smallest index if
 * several do):
 *   - a link between face-adjacent material sites is intact unless their side codes
 *     conflict (the blade sweep cut it); a directed link from a material site to an
 *     empty site or across a cut is a transition, with Hermite data (link midpoint,
 *     link direction outward);
 *   - each cube of 8 sites splits its material corners into local material regions
 *     (connected components of its intact edges); a region with a transition edge
 *     has one vertex, placed per axis at the mean coordinate of its transition
 *     midpoints along that axis (along all of them if none): local dual contouring;
 *   - one quad per directed transition through the vertices of its site's regions
 *     in the four cubes around the link, counter-clockwise seen from outside; a cut
 *     link gives one quad on each side (the two coincident faces of the cut);
 *   - vertex motion (one-way): fixed trilinear weights over its region's particles.
 * Vertices are ordered by cube (x fastest) and region (lowest corner); quads by site
 * (x fastest), axis x, y, z and outward +, -.
 * Device memory: a caller workspace.  tlmpm_surface_footprint gives the bytes of the
 * lattice tables (they depend on the grid only); tlmpm_surface_build counts the
 * vertices and quads in them, returns counts[2] = {vertices, quads} and the bytes
 * the whole surface needs in *needed, and fills the surface if the workspace holds
 * that many bytes (else TLMPM_E_NOMEM, counts and *needed still set: call again
 * with a workspace that large).  Both synchronise. */
tlmpm_status tlmpm_surface_footprint(tlmpm_scene* scene, size_t* bytes);
tlmpm_status tlmpm_surface_build(tlmpm_scene* scene, void* workspace, size_t bytes, int64_t counts[2],
                                 size_t* needed);

/* The built surface in workspace (the last tlmpm_surface_build of this scene):
 * x [nv][3] current vertex positions (the embedding in the current displacements),
 * X [nv][3] reference positions, code [nv] ternary side code of the vertex's region
 * (the union of its particles' digits), quads [nq][4] vertex indices, cut [nq] 1
 * for a quad on a cut face.  Any output may be NULL.  Synchronises. */
tlmpm_status tlmpm_surface_read(tlmpm_scene* scene, const void* workspace, size_t bytes, float* x, float* X,
                                uint64_t* code, int32_t* quads, uint8_t* cut);

/* ---- Batches: many independent scenes advanced by shared launches.
 * The substep is exactly that of tlmpm_step (Sec. III); a batch only groups the
 * kernel launches of its member scenes, so each kernel launch covers the work items
 * of every scene.  Results are bitwise those of stepping each scene alone with the
 * same tools.
 *   - Membership is fixed at creation.  While a batch is alive, its member scenes
 *     refuse every single-scene call (TLMPM_E_INVALID); tlmpm_batch_destroy
 *     synchronises and releases them.  A scene belongs to at most one batch.
 *   - Device memory: one caller workspace of tlmpm_batch_footprint() bytes (the
 *     per-scene parameter tables, the work-item lists and the per-call tool and
 *     wrench arrays), kept alive until tlmpm_batch_destroy.  The batch also holds a
 *     small pinned host staging area for the per-call tools.
 *   - Streams: creation synchronises the member scenes' streams; afterwards all work
 *     runs on the batch's stream. */
typedef struct tlmpm_batch tlmpm_batch; /* opaque */

#define TLMPM_MAX_TOOLS 4

/* Device bytes of a batch over these scenes (n_scenes >= 1, no repeats, none in a
 * live batch). */
tlmpm_status tlmpm_batch_footprint(tlmpm_scene* const* scenes, int32_t n_scenes, size_t* device_bytes);

/* Upper bound on the device bytes one scene of this description adds to a batch
 * workspace: for any set of such scenes, tlmpm_batch_footprint() is at most the sum
 * of their bounds.  For admission by device memory before the scene exists (a
 * server reserves tlmpm_scene_footprint() plus this for every running rollout). */
tlmpm_status tlmpm_batch_scene_bytes(const tlmpm_scene_desc* desc, size_t* device_bytes);

/* Build a batch.  Scenes whose pending deformation-gradient update was left in a
 * different slot-table state than the others first complete it alone. */
tlmpm_status tlmpm_batch_create(tlmpm_scene* const* scenes, int32_t n_scenes, void* dev_workspace, size_t bytes,
                                void* hip_stream, tlmpm_batch** out);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): tlmpm_batch_create
 * without a workspace argument.  The batch workspace is a fixed array of
 * TL_STATIC_SCRATCH_BYTES = 16 MiB in the library's device image, one per GPU
 * (the calling thread's current device, 0..7), held until the process ends; its
 * per-call tool staging is a static host array (pageable, so each tlmpm_batch_step
 * first waits for the batch's stream).  This call allocates no device or pinned
 * memory (no hipMalloc, hipHostMalloc, hipFree or torch allocator); the handle's
 * host bookkeeping is on the C++ heap.  A device's array serves one batch at a
 * time: while a batch built here is alive, another call on the same device fails
 * with TLMPM_E_INVALID (two batches on one array would race).  Nothing in the
 * array needs to start at zero: creation uploads the tables and every step
 * uploads its tools and clears its wrench sums.  TLMPM_E_NOMEM if the batch needs
 * more than 16 MiB (tlmpm_batch_footprint) or more than 1024 scenes; 256 scenes of
 * 13.3M particles need 3.2 MiB.  Otherwise as tlmpm_batch_create; destroy with
 * tlmpm_batch_destroy, which releases the array. */
tlmpm_status tlmpm_batch_create_static(tlmpm_scene* const* scenes, int32_t n_scenes, void* hip_stream,
                                       tlmpm_batch** out);

tlmpm_status tlmpm_batch_destroy(tlmpm_batch* batch);

/* n_substeps substeps of every member scene (as tlmpm_step).  tools: array of
 * n_scenes * TLMPM_MAX_TOOLS records; scene s uses tools[s * TLMPM_MAX_TOOLS + t]
 * for t < n_tools[s] (unused records are not read; tools may be NULL if every count
 * is 0).  wrench: NULL, or [n_scenes][TLMPM_MAX_TOOLS][6] averaged per scene as in
 * tlmpm_step (entries past a scene's tool count are 0); a non-NULL pointer
 * synchronises.  Invalid tools of any scene fail the call before any launch. */
tlmpm_status tlmpm_batch_step(tlmpm_batch* batch, const tlmpm_tool* tools, const int32_t* n_tools,
                              int32_t n_substeps, double* wrench);

/* Waits for the batch's queued work. */
tlmpm_status tlmpm_batch_sync(tlmpm_batch* batch);

/* HIP graph replay of the batch's substeps, as tlmpm_set_graphs. */
tlmpm_status tlmpm_batch_set_graphs(tlmpm_batch* batch, int32_t enable);

/* Kernel timing of the batch's launches, as tlmpm_profile_enable / _read. */
tlmpm_status tlmpm_batch_profile_enable(tlmpm_batch* batch, int32_t enable);
tlmpm_status tlmpm_batch_profile_read(tlmpm_batch* batch, int32_t n_classes, double* ms, int64_t* launches);

/* Text of the last error on the calling thread ("" if none). */
const char* tlmpm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TLMPM_H */
