/*
 * tlmpm_oracle.c -- plain FP64 CPU oracle for total-Lagrangian MPM cutting with
 * persistent ternary side labels (BladeMaster, arXiv 2609.27342).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the GPU
 * path is checked against.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product library never links or calls it.
 * It shares no code, header, table or constant with the HIP path.
 *
 * It is written for obviousness, not speed: array-of-structs state in FP64, a
 * scatter P2G into per-node linked lists of (code, state) accumulators, a brute
 * per-digit conflict test, linear scans.  Every function cites the passage of the
 * paper it follows.  Where the paper is silent the reading used is stated inline.
 *
 * Step order within one substep (Sec. III-B, III-D, III-E, App.):
 *   contact impulses on x^n, v^n, c^n -> label-masked P2G (Eq. 2) with gravity and
 *   contact impulses -> compatibility coupling (Eq. 8) -> grid update (Eq. 9) ->
 *   PIC/FLIP G2P of v and x (Eq. 17) -> MUSL re-scatter with the same coupling ->
 *   deformation-gradient update from the remapped velocities.
 *
 * Parity status of each part is recorded next to its function ("pinned by ..." or
 * "parity unpinned").
 *
 * Threads: loops whose iterations are independent (per particle or per node, each
 * writing only its own entries) may run under OpenMP; every sum over particles
 * (the scatter into node accumulators, the wrench) stays serial in particle order,
 * so the result does not depend on the thread count.  orc_set_threads selects it.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_CUTS 40
#define ORC_MAX_RIGID 17 /* floor + up to 16 tools */

enum { ORC_OK = 0, ORC_E_INVALID = 1, ORC_E_NONFINITE = 5 };

/* ------------------------------------------------------------------------- */
/* Public structs (mirrored by ctypes in oracle.py).                          */
/* ------------------------------------------------------------------------- */
typedef struct {
    double dx;
    double origin[3];
    int32_t cells[3];
    int32_t max_cuts;
    double dt;
    double gravity[3];
    double beta; /* PIC/FLIP blend of Eq. 17 */
    double nu;   /* Poisson ratio (E is per particle) */
    /* contact (Sec. III-E) */
    double s_R, s_n, gamma_k, gamma_c, mu_s, mu_d;
    int32_t material_contact;
    int32_t floor_on;
    double floor_z;
    /* cutting resistance (Eq. 5) */
    double G_c, zeta, u_min;
    int32_t single_field; /* negative control: every particle scatters to one logical grid */
    int32_t material;     /* 0 Neo-Hookean, 1 fixed-corotated (Sec. III-B) */
    double viscosity;     /* Newtonian viscosity eta (Pa s), 0 = none */
    double yield_stress;  /* von Mises yield stress (Pa), 0 = elastic */
    int32_t stencil;      /* 0 trilinear (8 nodes), 1 quadratic B-spline (27 nodes) */
    int32_t pad_;
} orc_params;

/* A blade record: the cut frame of Eq. 3 and the band extents of Eq. 4. */
typedef struct {
    int32_t cut_index; /* k: the ternary digit this blade assigns */
    int32_t new_cut;   /* start of cut k: reset D_p to zero (Sec. III-A) */
    double x_e[3];     /* point at the middle of the blade edge */
    double n[3];       /* cutting-plane normal */
    double e[3];       /* axis along the finite edge */
    double d[3];       /* front direction, pointing toward the cutting front */
    double v_e[3];     /* velocity of x_e */
    double half_len;   /* L_k */
    double half_width; /* h_k */
    double b_back;     /* rear extent of the band, also the blade height behind the edge */
    double b_lead;     /* lead extent of the band */
} orc_blade;

/* A kinematic rigid tool: a zero-thickness rectangle in the blade plane spanning
 * |l| <= half_len along e and -b_back <= f <= 0 along d (reading R18). */
typedef struct {
    orc_blade blade;
    double x_B[3];     /* reference point for the torque of Eq. 16 */
    double v_B[3];
    double omega_B[3];
    double w_B;        /* inverse effective mass, 0 for a prescribed tool */
    int32_t contact;   /* tool-material contact on */
    int32_t cutting;   /* directional contact work and release of Eq. 5 */
    double inv_mass;   /* a free rigid tool: 1/M ... */
    double inv_inertia[9]; /* ... and I^-1 about x_B in world axes (row major) */
} orc_tool;

/* ------------------------------------------------------------------------- */
/* Internal state.                                                            */
/* ------------------------------------------------------------------------- */
typedef struct node_entry {
    uint64_t code;
    double m;
    double p[3], dp[3];       /* P2G momentum and impulse (Eq. 2 plus external/contact) */
    double pbar[3], dpbar[3]; /* after coupling (Eq. 8) */
    double pt[3], ptbar[3];   /* MUSL re-scatter momentum before/after coupling */
    double vt[3];             /* remapped velocity */
    struct node_entry* next;
} node_entry;

typedef struct {
    long p, q;      /* p < q */
    double u[3];    /* tangential spring of the pair, oriented for p */
    double J[3];    /* impulse on p of the substep that stored this entry */
} pair_hist;

typedef struct orc_scene {
    orc_params P;
    long n;
    long nodes[3];
    double *X, *x, *v, *F; /* X,x,v: [n][3]; F: [n][9] row-major */
    double* Fdot;          /* [n][9] rate of F of the last update (viscosity) */
    double* Fpi;           /* [n][9] inverse plastic deformation gradient F_p^{-1} */
    double *vol0, *mass, *E;
    uint8_t* dig;          /* [n][max_cuts] ternary digits */
    double* D;             /* cutting progress */
    double* J;             /* contact impulse per particle, scratch */
    /* rigid contact history, per body slot and particle: u_t[3] and a live flag */
    double* rh_u;          /* [ORC_MAX_RIGID][n][3] */
    uint8_t* rh_live;      /* [ORC_MAX_RIGID][n] */
    /* material pair history, sorted by (p, q) */
    pair_hist* ph;
    long n_ph, cap_ph;
    /* grid: per-node list heads and an entry pool */
    node_entry** head;
    node_entry* pool;
    long n_pool, cap_pool;
    /* reference cell of every particle and a cell occupancy table (contact candidates) */
    long* cell_of;
    int32_t* cell_count;
    /* diagnostics of the last step */
    long last_pairs;
    long last_candidates;
    int status;
} orc_scene;

/* ------------------------------------------------------------------------- */
/* Small vector helpers.                                                      */
/* ------------------------------------------------------------------------- */
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double norm3(const double* a) { return sqrt(dot3(a, a)); }
static void cross3(const double* a, const double* b, double* c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* ------------------------------------------------------------------------- */
/* Ternary codes (Eq. 7) and the conflict predicate (Sec. III-D).             */
/* Pinned by the full digit-pair truth table and encode/decode round trips.   */
/* ------------------------------------------------------------------------- */
uint64_t orc_encode(const uint8_t* digits, int K)
{
    uint64_t c = 0, w = 1;
    for (int k = 0; k < K; k++) {
        c += (uint64_t)digits[k] * w;
        w *= 3;
    }
    return c;
}

int orc_digit(uint64_t code, int k)
{
    for (int i = 0; i < k; i++) code /= 3;
    return (int)(code % 3);
}

/* Two codes conflict iff some cut has digit 1 in one and 2 in the other. */
int orc_conflict(uint64_t a, uint64_t b, int K)
{
    for (int k = 0; k < K; k++) {
        int da = (int)(a % 3), db = (int)(b % 3);
        if ((da == 1 && db == 2) || (da == 2 && db == 1)) return 1;
        a /= 3;
        b /= 3;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Interpolation in the reference configuration (Eq. 1).                      */
/* Reading R1: trilinear hat (linear B-spline) over the 8 corners of the base  */
/* cell floor((X - origin)/dx); weights (1-t, t) and derivatives (-1/dx, 1/dx) */
/* per axis.  Reading R33 adds the quadratic B-spline over 27 nodes.  Pinned  */
/* by partition of unity, zero gradient sum, linear reproduction, the closed   */
/* form of each weight and finite differences of the weights.                  */
/* ------------------------------------------------------------------------- */
static int base_cell(const orc_params* P, const double* X, int* base, double* t)
{
    for (int a = 0; a < 3; a++) {
        double q = (X[a] - P->origin[a]) / P->dx;
        double b = floor(q);
        base[a] = (int)b;
        t[a] = q - b;
        if (base[a] < 0 || base[a] >= P->cells[a]) return -1;
    }
    return 0;
}

/* Quadratic B-spline of the node distance r (in cells): 3/4 - r^2 for |r| < 1/2,  */
/* (3/2 - |r|)^2 / 2 for 1/2 <= |r| < 3/2, else 0 (reading R33), and its derivative.*/
static double bspline2(double r)
{
    double a = fabs(r);
    if (a < 0.5) return 0.75 - a * a;
    if (a < 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
    return 0.0;
}

static double bspline2_d(double r)
{
    double a = fabs(r), sg = r < 0.0 ? -1.0 : 1.0;
    if (a < 0.5) return -2.0 * r;
    if (a < 1.5) return -sg * (1.5 - a);
    return 0.0;
}

/* 27-node stencil: the nodes base .. base + 2 per axis with base = floor(q - 1/2), */
/* q = (X - origin)/dx; each weight is the B-spline of the node's own distance.    */
static int shape_quadratic(const orc_params* P, const double* X, long* node, double* w, double* grad)
{
    int base[3];
    double q[3];
    for (int a = 0; a < 3; a++) {
        q[a] = (X[a] - P->origin[a]) / P->dx;
        base[a] = (int)floor(q[a] - 0.5);
        if (base[a] < 0 || base[a] + 2 > P->cells[a]) return -1;
    }
    long nx = P->cells[0] + 1, ny = P->cells[1] + 1;
    int k = 0;
    for (int c = 0; c < 3; c++)
        for (int b = 0; b < 3; b++)
            for (int a = 0; a < 3; a++, k++) {
                double rx = q[0] - (base[0] + a), ry = q[1] - (base[1] + b), rz = q[2] - (base[2] + c);
                double wx = bspline2(rx), wy = bspline2(ry), wz = bspline2(rz);
                w[k] = wx * wy * wz;
                grad[3 * k + 0] = bspline2_d(rx) / P->dx * wy * wz;
                grad[3 * k + 1] = wx * bspline2_d(ry) / P->dx * wz;
                grad[3 * k + 2] = wx * wy * bspline2_d(rz) / P->dx;
                if (node) node[k] = ((long)(base[2] + c) * ny + (base[1] + b)) * nx + (base[0] + a);
            }
    return 0;
}

/* Nodes of the stencil: 8 (trilinear) or 27 (quadratic B-spline). */
int orc_stencil_nodes(const orc_params* P) { return P->stencil == 1 ? 27 : 8; }

int orc_shape(const orc_params* P, const double* X, long* node, double* w, double* grad)
{
    if (P->stencil == 1) return shape_quadratic(P, X, node, w, grad);
    int base[3];
    double t[3];
    if (base_cell(P, X, base, t)) return -1;
    long nx = P->cells[0] + 1, ny = P->cells[1] + 1;
    int k = 0;
    for (int c = 0; c < 2; c++)
        for (int b = 0; b < 2; b++)
            for (int a = 0; a < 2; a++, k++) {
                double wx = a ? t[0] : 1.0 - t[0];
                double wy = b ? t[1] : 1.0 - t[1];
                double wz = c ? t[2] : 1.0 - t[2];
                double gx = (a ? 1.0 : -1.0) / P->dx;
                double gy = (b ? 1.0 : -1.0) / P->dx;
                double gz = (c ? 1.0 : -1.0) / P->dx;
                w[k] = wx * wy * wz;
                grad[3 * k + 0] = gx * wy * wz;
                grad[3 * k + 1] = wx * gy * wz;
                grad[3 * k + 2] = wx * wy * gz;
                if (node) node[k] = ((long)(base[2] + c) * ny + (base[1] + b)) * nx + (base[0] + a);
            }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Constitutive model (reading R2: compressible Neo-Hookean, the material the */
/* benchmark scenes name; the paper's fixed-corotated model is not used here). */
/*   psi = mu/2 (tr F^T F - 3) - mu ln J + lambda/2 (ln J)^2                    */
/*   P   = mu (F - F^{-T}) + lambda ln J F^{-T}                                 */
/* Pinned by P(I)=0, P(R)=0, objectivity, small-strain Hooke and finite        */
/* differences of psi.                                                         */
/* ------------------------------------------------------------------------- */
static double det3(const double* F)
{
    return F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
           F[2] * (F[3] * F[7] - F[4] * F[6]);
}

static void lame(double E, double nu, double* mu, double* lam)
{
    *mu = E / (2.0 * (1.0 + nu));
    *lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
}

/* Returns 0, or -1 if det F <= 0 (P left as NaN). */
int orc_neo_hookean_P(double E, double nu, const double* F, double* P)
{
    double mu, lam;
    lame(E, nu, &mu, &lam);
    double J = det3(F);
    if (!(J > 0.0)) {
        for (int i = 0; i < 9; i++) P[i] = NAN;
        return -1;
    }
    /* cofactor matrix: F^{-T} = cof(F) / J */
    double C[9];
    C[0] = F[4] * F[8] - F[5] * F[7];
    C[1] = F[5] * F[6] - F[3] * F[8];
    C[2] = F[3] * F[7] - F[4] * F[6];
    C[3] = F[2] * F[7] - F[1] * F[8];
    C[4] = F[0] * F[8] - F[2] * F[6];
    C[5] = F[1] * F[6] - F[0] * F[7];
    C[6] = F[1] * F[5] - F[2] * F[4];
    C[7] = F[2] * F[3] - F[0] * F[5];
    C[8] = F[0] * F[4] - F[1] * F[3];
    double lnJ = log(J);
    for (int i = 0; i < 9; i++) {
        double FiT = C[i] / J;
        P[i] = mu * (F[i] - FiT) + lam * lnJ * FiT;
    }
    return 0;
}

double orc_neo_hookean_psi(double E, double nu, const double* F)
{
    double mu, lam;
    lame(E, nu, &mu, &lam);
    double J = det3(F);
    double tr = 0.0;
    for (int i = 0; i < 9; i++) tr += F[i] * F[i];
    double lnJ = log(J);
    return 0.5 * mu * (tr - 3.0) - mu * lnJ + 0.5 * lam * lnJ * lnJ;
}

/* ------------------------------------------------------------------------- */
/* Fixed-corotated elasticity and Newtonian viscosity (Sec. III-B names them   */
/* as the paper's material model; reading R31).                                */
/* ------------------------------------------------------------------------- */
/* Eigen-decomposition A = Q diag(lam) Q^T of a symmetric 3x3 matrix by cyclic  */
/* Jacobi rotations (columns of Q are the eigenvectors).                       */
static void sym_eig3(const double* A_in, double* lam, double* Q)
{
    double A[9];
    memcpy(A, A_in, sizeof(A));
    for (int i = 0; i < 9; i++) Q[i] = (i % 4 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 60; sweep++) {
        double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
        double tot = off;
        for (int i = 0; i < 3; i++) tot += A[4 * i] * A[4 * i];
        if (off <= 1e-32 * tot || off == 0.0) break;
        for (int pq = 0; pq < 3; pq++) {
            int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
            double apq = A[3 * p + q];
            if (apq == 0.0) continue;
            /* rotation angle that zeroes A[p][q] */
            double theta = (A[3 * q + q] - A[3 * p + p]) / (2.0 * apq);
            double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
            /* A <- G^T A G, Q <- Q G with G the rotation in the (p, q) plane */
            for (int k = 0; k < 3; k++) {
                double akp = A[3 * k + p], akq = A[3 * k + q];
                A[3 * k + p] = c * akp - sn * akq;
                A[3 * k + q] = sn * akp + c * akq;
            }
            for (int k = 0; k < 3; k++) {
                double apk = A[3 * p + k], aqk = A[3 * q + k];
                A[3 * p + k] = c * apk - sn * aqk;
                A[3 * q + k] = sn * apk + c * aqk;
            }
            for (int k = 0; k < 3; k++) {
                double qkp = Q[3 * k + p], qkq = Q[3 * k + q];
                Q[3 * k + p] = c * qkp - sn * qkq;
                Q[3 * k + q] = sn * qkp + c * qkq;
            }
        }
    }
    for (int i = 0; i < 3; i++) lam[i] = A[4 * i];
}

/* Polar decomposition F = R S with S = (F^T F)^{1/2} symmetric positive       */
/* definite and R = F S^{-1} a rotation (det F > 0).  Returns -1 otherwise.   */
int orc_polar(const double* F, double* R, double* S)
{
    if (!(det3(F) > 0.0)) return -1;
    double C[9], lam[3], Q[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double a = 0.0;
            for (int k = 0; k < 3; k++) a += F[3 * k + i] * F[3 * k + j];
            C[3 * i + j] = a;
        }
    sym_eig3(C, lam, Q);
    double Si[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double a = 0.0, b = 0.0;
            for (int k = 0; k < 3; k++) {
                a += Q[3 * i + k] * sqrt(lam[k]) * Q[3 * j + k];
                b += Q[3 * i + k] / sqrt(lam[k]) * Q[3 * j + k];
            }
            S[3 * i + j] = a;
            Si[3 * i + j] = b;
        }
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double a = 0.0;
            for (int k = 0; k < 3; k++) a += F[3 * i + k] * Si[3 * k + j];
            R[3 * i + j] = a;
        }
    return 0;
}

static void cofactor3(const double* F, double* C)
{
    C[0] = F[4] * F[8] - F[5] * F[7];
    C[1] = F[5] * F[6] - F[3] * F[8];
    C[2] = F[3] * F[7] - F[4] * F[6];
    C[3] = F[2] * F[7] - F[1] * F[8];
    C[4] = F[0] * F[8] - F[2] * F[6];
    C[5] = F[1] * F[6] - F[0] * F[7];
    C[6] = F[1] * F[5] - F[2] * F[4];
    C[7] = F[2] * F[3] - F[0] * F[5];
    C[8] = F[0] * F[4] - F[1] * F[3];
}

/* Fixed-corotated first Piola-Kirchhoff stress P = 2 mu (F - R) + lambda (J - 1) */
/* J F^{-T}, the derivative of psi = mu |F - R|^2 + lambda/2 (J - 1)^2.          */
int orc_fcr_P(double E, double nu, const double* F, double* P)
{
    double mu, lam, R[9], S[9], C[9];
    lame(E, nu, &mu, &lam);
    if (orc_polar(F, R, S)) {
        for (int i = 0; i < 9; i++) P[i] = NAN;
        return -1;
    }
    double J = det3(F);
    cofactor3(F, C); /* J F^{-T} */
    for (int i = 0; i < 9; i++) P[i] = 2.0 * mu * (F[i] - R[i]) + lam * (J - 1.0) * C[i];
    return 0;
}

double orc_fcr_psi(double E, double nu, const double* F)
{
    double mu, lam, R[9], S[9];
    lame(E, nu, &mu, &lam);
    if (orc_polar(F, R, S)) return NAN;
    double a = 0.0;
    for (int i = 0; i < 9; i++) a += (F[i] - R[i]) * (F[i] - R[i]);
    double J = det3(F);
    return mu * a + 0.5 * lam * (J - 1.0) * (J - 1.0);
}

static void matmul3(const double* A, const double* B, double* C)
{
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double a = 0.0;
            for (int k = 0; k < 3; k++) a += A[3 * i + k] * B[3 * k + j];
            C[3 * i + j] = a;
        }
}

/* von Mises projection of an elastic deformation gradient (reading R32): with    */
/* F_e = U diag(sigma) V^T and Hencky strain eps = ln sigma, the deviatoric part   */
/* of the Kirchhoff stress of the logarithmic model, 2 mu dev(eps), is scaled back */
/* onto the cylinder |2 mu dev(eps)| = sqrt(2/3) sigma_y; the volumetric part is   */
/* kept.  Writes the projected F_e; returns 1 if it yielded, 0 if not, -1 if det  */
/* F_e <= 0.                                                                       */
int orc_vm_project(double E, double nu, double sigma_y, const double* Fe, double* Fe_new)
{
    double mu, lam;
    lame(E, nu, &mu, &lam);
    memcpy(Fe_new, Fe, sizeof(double) * 9);
    if (!(det3(Fe) > 0.0)) return -1;
    double C[9], ev[3], V[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double a = 0.0;
            for (int k = 0; k < 3; k++) a += Fe[3 * k + i] * Fe[3 * k + j];
            C[3 * i + j] = a;
        }
    sym_eig3(C, ev, V);
    double sg[3], eps[3];
    for (int k = 0; k < 3; k++) {
        sg[k] = sqrt(ev[k]);
        eps[k] = log(sg[k]);
    }
    double tr = (eps[0] + eps[1] + eps[2]) / 3.0, dev[3], nd = 0.0;
    for (int k = 0; k < 3; k++) {
        dev[k] = eps[k] - tr;
        nd += dev[k] * dev[k];
    }
    nd = sqrt(nd);
    const double lim = sqrt(2.0 / 3.0) * sigma_y;
    if (!(2.0 * mu * nd > lim)) return 0;
    const double scale = lim / (2.0 * mu * nd);
    /* U = F_e V diag(1/sigma); F_e_new = U diag(exp(eps_new)) V^T */
    double U[9];
    for (int i = 0; i < 3; i++)
        for (int k = 0; k < 3; k++) {
            double a = 0.0;
            for (int j = 0; j < 3; j++) a += Fe[3 * i + j] * V[3 * j + k];
            U[3 * i + k] = a / sg[k];
        }
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double a = 0.0;
            for (int k = 0; k < 3; k++) a += U[3 * i + k] * exp(tr + scale * dev[k]) * V[3 * j + k];
            Fe_new[3 * i + j] = a;
        }
    return 1;
}

static int inv3(const double* A, double* Ai)
{
    double C[9], d = det3(A);
    if (d == 0.0) return -1;
    cofactor3(A, C);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) Ai[3 * i + j] = C[3 * j + i] / d;
    return 0;
}

/* Newtonian viscous first Piola-Kirchhoff stress: Cauchy stress eta (l + l^T)   */
/* with l = Fdot F^{-1} the spatial velocity gradient, pulled back by J F^{-T}.  */
int orc_visc_P(double eta, const double* F, const double* Fdot, double* P)
{
    double J = det3(F), C[9];
    if (!(J > 0.0)) {
        for (int i = 0; i < 9; i++) P[i] = NAN;
        return -1;
    }
    cofactor3(F, C); /* J F^{-T}; F^{-1} = C^T / J */
    double l[9], sg[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double a = 0.0;
            for (int k = 0; k < 3; k++) a += Fdot[3 * i + k] * C[3 * j + k] / J;
            l[3 * i + j] = a;
        }
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) sg[3 * i + j] = eta * (l[3 * i + j] + l[3 * j + i]);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double a = 0.0;
            for (int k = 0; k < 3; k++) a += sg[3 * i + k] * C[3 * k + j];
            P[3 * i + j] = a;
        }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Compatibility coupling at one node (Eq. 8).                                */
/* S logical grids with masses m[a], codes[a] and a 3-vector field f[a]; the   */
/* output is f_bar[a] = f[a] + (1/M) sum_{b != a, compatible} (m_a f_b - m_b f_a)*/
/* with M the sum of ALL masses at the node (reading R6), using pre-exchange    */
/* values only.  Pinned by the all-compatible, all-conflicting and {0,1,2}      */
/* closed forms and the antisymmetry sum.                                       */
/* ------------------------------------------------------------------------- */
void orc_couple(int S, const double* m, const uint64_t* codes, int K, const double* f, double* fbar)
{
    double M = 0.0;
    for (int a = 0; a < S; a++) M += m[a];
    for (int a = 0; a < S; a++) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int b = 0; b < S; b++) {
            if (b == a) continue;
            if (orc_conflict(codes[a], codes[b], K)) continue;
            for (int j = 0; j < 3; j++) acc[j] += m[a] * f[3 * b + j] - m[b] * f[3 * a + j];
        }
        for (int j = 0; j < 3; j++) fbar[3 * a + j] = f[3 * a + j] + (M > 0.0 ? acc[j] / M : 0.0);
    }
}

/* ------------------------------------------------------------------------- */
/* Side-label assignment (Eqs. 3, 4, 6).                                       */
/* Reading R11: the predicates are evaluated in FP64 with a fixed evaluation   */
/* order and no fused multiply-add, so a caller that feeds FP32 state widened  */
/* to FP64 obtains a deterministic answer:                                     */
/*   r = x - x_e;  s = (r0 n0 + r1 n1) + r2 n2  (likewise l, f)                */
/*   u_c = ((ve0-v0) d0 + (ve1-v1) d1) + (ve2-v2) d2                            */
/*   band: |s| <= h, |l| <= L, -b_back - max(u_c dt, 0) <= f <= b_lead          */
/*   assign when in band, f <= 0 and the digit is 0: 1 if s < 0 else 2 (R8).   */
/* Returns the new digit (0 if unchanged).  Pinned by hand cases and geometric */
/* brute force in the tests.                                                    */
/* ------------------------------------------------------------------------- */
int orc_label_digit(const double* x, const double* v, const orc_blade* B, double dt, int digit_now)
{
    if (digit_now != 0) return 0; /* persistence: nonzero digits never change */
    /* this file is compiled with -ffp-contract=off: every product is rounded */
    double r0 = x[0] - B->x_e[0], r1 = x[1] - B->x_e[1], r2 = x[2] - B->x_e[2];
    double s = (r0 * B->n[0] + r1 * B->n[1]) + r2 * B->n[2];
    double l = (r0 * B->e[0] + r1 * B->e[1]) + r2 * B->e[2];
    double f = (r0 * B->d[0] + r1 * B->d[1]) + r2 * B->d[2];
    double uc = ((B->v_e[0] - v[0]) * B->d[0] + (B->v_e[1] - v[1]) * B->d[1]) + (B->v_e[2] - v[2]) * B->d[2];
    double lo = -B->b_back - fmax(uc * dt, 0.0);
    int in_band = fabs(s) <= B->half_width && fabs(l) <= B->half_len && lo <= f && f <= B->b_lead;
    if (!in_band || !(f <= 0.0)) return 0;
    return (s < 0.0) ? 1 : 2;
}

/* Threads of the loops with independent iterations (see the file header). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_get_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------- */
/* Scene lifetime.                                                            */
/* ------------------------------------------------------------------------- */
void orc_destroy(orc_scene* s)
{
    if (!s) return;
    free(s->X);
    free(s->x);
    free(s->v);
    free(s->F);
    free(s->Fdot);
    free(s->Fpi);
    free(s->vol0);
    free(s->mass);
    free(s->E);
    free(s->dig);
    free(s->D);
    free(s->J);
    free(s->rh_u);
    free(s->rh_live);
    free(s->ph);
    free(s->head);
    free(s->pool);
    free(s->cell_of);
    free(s->cell_count);
    free(s);
}

orc_scene* orc_create(const orc_params* P, long n, const double* X, const double* v0, const double* vol0,
                      const double* mass, const double* E)
{
    if (!P || n < 0 || P->max_cuts < 0 || P->max_cuts > ORC_MAX_CUTS || !(P->dx > 0.0)) return NULL;
    orc_scene* s = (orc_scene*)calloc(1, sizeof(orc_scene));
    s->P = *P;
    s->n = n;
    for (int a = 0; a < 3; a++) s->nodes[a] = P->cells[a] + 1;
    long nn = s->nodes[0] * s->nodes[1] * s->nodes[2];
    long nc = (long)P->cells[0] * P->cells[1] * P->cells[2];
    long K = P->max_cuts > 0 ? P->max_cuts : 1;
    s->X = (double*)malloc(sizeof(double) * 3 * (n + 1));
    s->x = (double*)malloc(sizeof(double) * 3 * (n + 1));
    s->v = (double*)calloc(3 * (n + 1), sizeof(double));
    s->F = (double*)malloc(sizeof(double) * 9 * (n + 1));
    s->Fdot = (double*)calloc(9 * (n + 1), sizeof(double));
    s->Fpi = (double*)calloc(9 * (n + 1), sizeof(double));
    for (long p = 0; p < n; p++)
        for (int i = 0; i < 3; i++) s->Fpi[9 * p + 4 * i] = 1.0;
    s->vol0 = (double*)malloc(sizeof(double) * (n + 1));
    s->mass = (double*)malloc(sizeof(double) * (n + 1));
    s->E = (double*)malloc(sizeof(double) * (n + 1));
    s->dig = (uint8_t*)calloc((size_t)(n + 1) * K, 1);
    s->D = (double*)calloc(n + 1, sizeof(double));
    s->J = (double*)calloc(3 * (n + 1), sizeof(double));
    s->rh_u = (double*)calloc((size_t)ORC_MAX_RIGID * 3 * (n + 1), sizeof(double));
    s->rh_live = (uint8_t*)calloc((size_t)ORC_MAX_RIGID * (n + 1), 1);
    s->head = (node_entry**)calloc(nn, sizeof(node_entry*));
    s->cell_of = (long*)malloc(sizeof(long) * (n + 1));
    s->cell_count = (int32_t*)calloc(nc > 0 ? nc : 1, sizeof(int32_t));
    for (long p = 0; p < n; p++) {
        int base[3];
        double t[3];
        for (int a = 0; a < 3; a++) s->X[3 * p + a] = s->x[3 * p + a] = X[3 * p + a];
        long nd[27];
        double wq[27], gq[81];
        if (base_cell(P, &s->X[3 * p], base, t) || orc_shape(P, &s->X[3 * p], nd, wq, gq)) {
            orc_destroy(s);
            return NULL;
        }
        s->cell_of[p] = ((long)base[2] * P->cells[1] + base[1]) * P->cells[0] + base[0];
        s->cell_count[s->cell_of[p]]++;
        if (v0)
            for (int a = 0; a < 3; a++) s->v[3 * p + a] = v0[3 * p + a];
        for (int i = 0; i < 9; i++) s->F[9 * p + i] = (i % 4 == 0) ? 1.0 : 0.0;
        s->vol0[p] = vol0[p];
        s->mass[p] = mass[p];
        s->E[p] = E[p];
    }
    return s;
}

/* Raw access for the test harness (shared-input comparisons and rollouts). */
void orc_get(const orc_scene* s, double* x, double* v, double* F, uint8_t* dig, double* D)
{
    long n = s->n, K = s->P.max_cuts;
    if (x) memcpy(x, s->x, sizeof(double) * 3 * n);
    if (v) memcpy(v, s->v, sizeof(double) * 3 * n);
    if (F) memcpy(F, s->F, sizeof(double) * 9 * n);
    if (dig && K) memcpy(dig, s->dig, (size_t)n * K);
    if (D) memcpy(D, s->D, sizeof(double) * n);
}

void orc_set(orc_scene* s, const double* x, const double* v, const double* F, const uint8_t* dig, const double* D)
{
    long n = s->n, K = s->P.max_cuts;
    if (x) memcpy(s->x, x, sizeof(double) * 3 * n);
    if (v) memcpy(s->v, v, sizeof(double) * 3 * n);
    if (F) memcpy(s->F, F, sizeof(double) * 9 * n);
    if (dig && K) memcpy(s->dig, dig, (size_t)n * K);
    if (D) memcpy(s->D, D, sizeof(double) * n);
}

long orc_last_pairs(const orc_scene* s) { return s->last_pairs; }
long orc_last_candidates(const orc_scene* s) { return s->last_candidates; }

static uint64_t code_of(const orc_scene* s, long p)
{
    if (s->P.single_field) return 0;
    return orc_encode(&s->dig[(size_t)p * s->P.max_cuts], s->P.max_cuts);
}

/* Label pass over arrays: positions x [n][3], velocities v [n][3] and digits    */
/* dig [n][K], updated in place for each blade in turn.  Returns the number of    */
/* digits set, or -1 for a cut index outside [0, K).                              */
long orc_label_pass(long n, const double* x, const double* v, uint8_t* dig, int K, const orc_blade* blades,
                    int nb, double dt)
{
    long changed = 0;
    for (int b = 0; b < nb; b++) {
        const orc_blade* B = &blades[b];
        if (B->cut_index < 0 || B->cut_index >= K) return -1;
#pragma omp parallel for reduction(+ : changed)
        for (long p = 0; p < n; p++) {
            uint8_t* dg = &dig[(size_t)p * K + B->cut_index];
            int nd = orc_label_digit(&x[3 * p], &v[3 * p], B, dt, *dg);
            if (nd) {
                *dg = (uint8_t)nd;
                changed++;
            }
        }
    }
    return changed;
}

/* Label pass of a scene on its stored x^n, v^n.  A new cut first resets D to     */
/* zero for every particle (Sec. III-A).  Returns the number of digits set.        */
long orc_assign_labels(orc_scene* s, const orc_blade* blades, int nb)
{
    for (int b = 0; b < nb; b++)
        if (blades[b].new_cut)
            for (long p = 0; p < s->n; p++) s->D[p] = 0.0;
    return orc_label_pass(s->n, s->x, s->v, s->dig, s->P.max_cuts, blades, nb, s->P.dt);
}

/* ------------------------------------------------------------------------- */
/* History-based Coulomb friction (Eq. 12, reading R16).                      */
/* Input: relative velocity v_rel, unit normal nrm, normal force fn > 0,      */
/* effective mass meff and the stored spring u (updated in place).            */
/* Output: tangential force ft.                                               */
/* ------------------------------------------------------------------------- */
static void friction(const orc_params* P, const double* vrel, const double* nrm, double fn, double meff,
                     double* u, double* ft)
{
    double dt = P->dt;
    /* transport the stored spring to the current tangent plane, keeping its length */
    double un = dot3(u, nrm);
    double up[3] = {u[0] - un * nrm[0], u[1] - un * nrm[1], u[2] - un * nrm[2]};
    double lu = norm3(u), lp = norm3(up);
    double ut[3] = {0.0, 0.0, 0.0};
    if (lp > 0.0)
        for (int j = 0; j < 3; j++) ut[j] = up[j] * (lu / lp);
    double vn = dot3(vrel, nrm);
    double vt[3] = {vrel[0] - vn * nrm[0], vrel[1] - vn * nrm[1], vrel[2] - vn * nrm[2]};
    double kt = P->gamma_k * meff / (dt * dt);
    double ct = 2.0 * P->gamma_c * sqrt(meff * kt);
    double ftr[3];
    for (int j = 0; j < 3; j++) ftr[j] = -kt * ut[j] - ct * vt[j];
    double lf = norm3(ftr);
    if (lf <= P->mu_s * fn) {
        for (int j = 0; j < 3; j++) {
            ft[j] = ftr[j];
            u[j] = ut[j] + dt * vt[j];
        }
    } else {
        for (int j = 0; j < 3; j++) {
            ft[j] = P->mu_d * fn * ftr[j] / lf;
            u[j] = -(ft[j] + ct * vt[j]) / kt;
        }
    }
}

/* Contact radius of the spherical proxy (Sec. III-E): R = s_R V0^{1/3} / 2. */
static double radius(const orc_scene* s, long p) { return s->P.s_R * cbrt(s->vol0[p]) * 0.5; }

/* ------------------------------------------------------------------------- */
/* Tool-material contact (Eqs. 14-16) and directional contact work (Eq. 5).   */
/* body == 0 is the floor half-space z >= floor_z with outward normal +z;      */
/* body >= 1 is tools[body-1], a zero-thickness rectangle (reading R18).       */
/* Adds the impulse to s->J and the reaction to wrench[6] (if non-NULL).       */
/* Pinned by the inclined-plane stick/slip closed form, the one-step normal    */
/* response and the wrench balance in the tests.                               */
/* ------------------------------------------------------------------------- */
static void rigid_contact(orc_scene* s, int body, const orc_tool* T, double* wrench, const double* D_start)
{
    const orc_params* P = &s->P;
    double dt = P->dt;
    /* per-particle reactions, summed in particle order after the loop */
    double* wb = wrench ? (double*)malloc(sizeof(double) * 6 * (s->n + 1)) : NULL;
    uint8_t* wf = wrench ? (uint8_t*)calloc(s->n + 1, 1) : NULL;
#pragma omp parallel for
    for (long p = 0; p < s->n; p++) {
        const double* x = &s->x[3 * p];
        const double* v = &s->v[3 * p];
        double xc[3], nB[3], xB[3] = {0, 0, 0}, vB[3] = {0, 0, 0}, wB[3] = {0, 0, 0}, invm = 0.0;
        double R = radius(s, p), phi;
        if (body == 0) {
            xc[0] = x[0];
            xc[1] = x[1];
            xc[2] = P->floor_z;
            nB[0] = 0.0;
            nB[1] = 0.0;
            nB[2] = 1.0;
            phi = (x[2] - P->floor_z) - R;
            xB[0] = xc[0];
            xB[1] = xc[1];
            xB[2] = xc[2];
        } else {
            const orc_blade* B = &T->blade;
            double r[3] = {x[0] - B->x_e[0], x[1] - B->x_e[1], x[2] - B->x_e[2]};
            double al = dot3(r, B->e), be = -dot3(r, B->d);
            if (al < -B->half_len) al = -B->half_len;
            if (al > B->half_len) al = B->half_len;
            if (be < 0.0) be = 0.0;
            if (be > B->b_back) be = B->b_back;
            for (int j = 0; j < 3; j++) xc[j] = B->x_e[j] + al * B->e[j] - be * B->d[j];
            double df[3] = {x[0] - xc[0], x[1] - xc[1], x[2] - xc[2]};
            double dist = norm3(df);
            if (dist > 0.0)
                for (int j = 0; j < 3; j++) nB[j] = df[j] / dist;
            else
                for (int j = 0; j < 3; j++) nB[j] = B->n[j];
            phi = dist - R;
            for (int j = 0; j < 3; j++) {
                xB[j] = T->x_B[j];
                vB[j] = T->v_B[j];
                wB[j] = T->omega_B[j];
            }
        }
        /* relative velocity at the contact point and predicted gap (Eq. 14) */
        double arm[3] = {xc[0] - xB[0], xc[1] - xB[1], xc[2] - xB[2]}, wxr[3];
        if (body > 0) {
            /* inverse effective mass of the tool at x_c along n_B (Sec. III-E, Eq. 15):
             * the normal velocity change of the contact point per unit normal
             * impulse, 1/M + (r x n) . I^-1 (r x n), plus a given constant part */
            double rn[3], Irn[3];
            cross3(arm, nB, rn);
            for (int i = 0; i < 3; i++)
                Irn[i] = T->inv_inertia[3 * i] * rn[0] + T->inv_inertia[3 * i + 1] * rn[1] +
                         T->inv_inertia[3 * i + 2] * rn[2];
            invm = T->w_B + T->inv_mass + dot3(rn, Irn);
        }
        cross3(wB, arm, wxr);
        double vrel[3] = {v[0] - (vB[0] + wxr[0]), v[1] - (vB[1] + wxr[1]), v[2] - (vB[2] + wxr[2])};
        double vrn = dot3(vrel, nB);
        double phihat = phi + dt * fmin(vrn, 0.0);
        double meff = 1.0 / (1.0 / s->mass[p] + invm);
        double Jn = P->s_n * meff / dt * fmax(-phihat, 0.0); /* Eq. 15 */
        double* u = &s->rh_u[((size_t)body * s->n + p) * 3];
        uint8_t* live = &s->rh_live[(size_t)body * s->n + p];
        if (!(Jn > 0.0)) {
            u[0] = u[1] = u[2] = 0.0;
            *live = 0;
            continue;
        }
        if (!*live) u[0] = u[1] = u[2] = 0.0;
        double ft[3];
        friction(P, vrel, nB, Jn / dt, meff, u, ft);
        *live = 1;
        double JpB[3];
        for (int j = 0; j < 3; j++) JpB[j] = Jn * nB[j] + ft[j] * dt;
        /* directional contact work in the front band (Eq. 5, reading R13) */
        if (body > 0 && T->cutting) {
            const orc_blade* B = &T->blade;
            double r[3] = {x[0] - B->x_e[0], x[1] - B->x_e[1], x[2] - B->x_e[2]};
            double sv = dot3(r, B->n), lv = dot3(r, B->e), fv = dot3(r, B->d);
            double dv[3] = {B->v_e[0] - v[0], B->v_e[1] - v[1], B->v_e[2] - v[2]};
            double uc = dot3(dv, B->d);
            if (fabs(sv) <= B->half_width && fabs(lv) <= B->half_len && fv >= 0.0 && fv <= B->b_lead &&
                uc > P->u_min) {
                double Jc = fmax(dot3(JpB, B->d), 0.0);
                if (D_start[p] < 1.0) {
                    double Wth = P->G_c * pow(s->vol0[p], 2.0 / 3.0) * (1.0 - P->zeta) / P->zeta;
                    double Dn = s->D[p] + Jc * uc / Wth;
                    s->D[p] = Dn < 1.0 ? Dn : 1.0;
                } else {
                    for (int j = 0; j < 3; j++) JpB[j] -= Jc * B->d[j];
                }
            }
        }
        for (int j = 0; j < 3; j++) s->J[3 * p + j] += JpB[j];
        if (wrench) {
            double Fb[3] = {-JpB[0] / dt, -JpB[1] / dt, -JpB[2] / dt}, tq[3];
            cross3(arm, Fb, tq);
            for (int j = 0; j < 3; j++) {
                wb[6 * p + j] = Fb[j];
                wb[6 * p + 3 + j] = tq[j];
            }
            wf[p] = 1;
        }
    }
    if (wrench) {
        for (long p = 0; p < s->n; p++)
            if (wf[p])
                for (int j = 0; j < 6; j++) wrench[j] += wb[6 * p + j];
        free(wb);
        free(wf);
    }
}

/* ------------------------------------------------------------------------- */
/* Material-material contact (Eqs. 10-13).                                    */
/* Candidates (reading R17): a particle whose 3x3x3 block of reference cells   */
/* holds an empty or out-of-grid cell, or a particle whose code conflicts with */
/* its own.  A candidate pair is excluded when the reference cells differ by at*/
/* most one per axis and the codes are compatible.  Pairs are found by binning */
/* current positions with a bin edge no smaller than the largest reach.        */
/* Pinned by brute force over all candidate pairs and by the head-on closed    */
/* form in the tests.                                                          */
/* ------------------------------------------------------------------------- */
static int cmp_long2(const void* a, const void* b)
{
    const long* x = (const long*)a;
    const long* y = (const long*)b;
    if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
    return (x[1] > y[1]) - (x[1] < y[1]);
}

static int cmp_pair(const void* a, const void* b)
{
    const pair_hist* x = (const pair_hist*)a;
    const pair_hist* y = (const pair_hist*)b;
    if (x->p != y->p) return x->p < y->p ? -1 : 1;
    return (x->q > y->q) - (x->q < y->q);
}

static void cell_ijk(const orc_scene* s, long c, int* ijk)
{
    ijk[0] = (int)(c % s->P.cells[0]);
    ijk[1] = (int)((c / s->P.cells[0]) % s->P.cells[1]);
    ijk[2] = (int)(c / ((long)s->P.cells[0] * s->P.cells[1]));
}

/* cand[p] = 1 if particle p is a contact candidate. */
void orc_candidates(const orc_scene* s, uint8_t* cand)
{
    const orc_params* P = &s->P;
    long nc = (long)P->cells[0] * P->cells[1] * P->cells[2];
    /* per cell: list of particles, for the conflict test */
    long* start = (long*)calloc(nc + 1, sizeof(long));
    long* list = (long*)malloc(sizeof(long) * (s->n + 1));
    for (long p = 0; p < s->n; p++) start[s->cell_of[p] + 1]++;
    for (long c = 0; c < nc; c++) start[c + 1] += start[c];
    long* fill = (long*)malloc(sizeof(long) * (nc + 1));
    memcpy(fill, start, sizeof(long) * (nc + 1));
    for (long p = 0; p < s->n; p++) list[fill[s->cell_of[p]]++] = p;
#pragma omp parallel for
    for (long p = 0; p < s->n; p++) {
        int ijk[3];
        cell_ijk(s, s->cell_of[p], ijk);
        uint64_t cp = code_of(s, p);
        int is = 0;
        for (int dz = -1; dz <= 1 && !is; dz++)
            for (int dy = -1; dy <= 1 && !is; dy++)
                for (int dx = -1; dx <= 1 && !is; dx++) {
                    int a = ijk[0] + dx, b = ijk[1] + dy, c = ijk[2] + dz;
                    if (a < 0 || b < 0 || c < 0 || a >= P->cells[0] || b >= P->cells[1] || c >= P->cells[2]) {
                        is = 1;
                        break;
                    }
                    long cc = ((long)c * P->cells[1] + b) * P->cells[0] + a;
                    if (s->cell_count[cc] == 0) {
                        is = 1;
                        break;
                    }
                    for (long i = start[cc]; i < start[cc + 1]; i++)
                        if (orc_conflict(cp, code_of(s, list[i]), P->max_cuts)) {
                            is = 1;
                            break;
                        }
                }
        cand[p] = (uint8_t)is;
    }
    free(start);
    free(list);
    free(fill);
}

static int excluded(const orc_scene* s, long p, long q)
{
    int a[3], b[3];
    cell_ijk(s, s->cell_of[p], a);
    cell_ijk(s, s->cell_of[q], b);
    int near = abs(a[0] - b[0]) <= 1 && abs(a[1] - b[1]) <= 1 && abs(a[2] - b[2]) <= 1;
    return near && !orc_conflict(code_of(s, p), code_of(s, q), s->P.max_cuts);
}

static const pair_hist* find_hist(const orc_scene* s, long p, long q)
{
    long lo = 0, hi = s->n_ph - 1;
    while (lo <= hi) {
        long mid = (lo + hi) / 2;
        const pair_hist* h = &s->ph[mid];
        if (h->p == p && h->q == q) return h;
        if (h->p < p || (h->p == p && h->q < q))
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return NULL;
}

/* Evaluate one candidate pair p < q; returns 1 and fills J (impulse on p) and
 * the new history if the pair is in contact. */
static int pair_impulse(const orc_scene* s, long p, long q, double* Jpq, double* unew)
{
    const orc_params* P = &s->P;
    double dt = P->dt;
    const double *xp = &s->x[3 * p], *xq = &s->x[3 * q], *vp = &s->v[3 * p], *vq = &s->v[3 * q];
    double dx[3] = {xp[0] - xq[0], xp[1] - xq[1], xp[2] - xq[2]};
    double dist = norm3(dx);
    if (!(dist > 0.0)) return 0;
    double nrm[3] = {dx[0] / dist, dx[1] / dist, dx[2] / dist};
    double vrel[3] = {vp[0] - vq[0], vp[1] - vq[1], vp[2] - vq[2]};
    double vn = dot3(vrel, nrm);
    double dhat = radius(s, p) + radius(s, q) - (dist + fmin(dt * vn, 0.0)); /* Eq. 10 */
    double meff = s->mass[p] * s->mass[q] / (s->mass[p] + s->mass[q]);
    double fn = P->s_n * meff / (dt * dt) * fmax(dhat, 0.0); /* Eq. 11 */
    if (!(fn > 0.0)) return 0;
    const pair_hist* h = find_hist(s, p, q);
    double u[3] = {0.0, 0.0, 0.0};
    if (h)
        for (int j = 0; j < 3; j++) u[j] = h->u[j];
    double ft[3];
    friction(P, vrel, nrm, fn, meff, u, ft);
    for (int j = 0; j < 3; j++) {
        Jpq[j] = (fn * nrm[j] + ft[j]) * dt;
        unew[j] = u[j];
    }
    return 1;
}

static void push_pair(pair_hist** arr, long* n, long* cap, long p, long q, const double* u, const double* J)
{
    if (*n == *cap) {
        *cap = *cap ? 2 * *cap : 1024;
        *arr = (pair_hist*)realloc(*arr, sizeof(pair_hist) * *cap);
    }
    pair_hist* h = &(*arr)[(*n)++];
    h->p = p;
    h->q = q;
    for (int j = 0; j < 3; j++) {
        h->u[j] = u[j];
        h->J[j] = J[j];
    }
}

/* brute != 0: test every candidate pair (O(C^2)); else bin current positions. */
static void material_contact(orc_scene* s, int brute)
{
    uint8_t* cand = (uint8_t*)malloc(s->n + 1);
    orc_candidates(s, cand);
    long C = 0;
    for (long p = 0; p < s->n; p++) C += cand[p];
    s->last_candidates = C;
    long* ids = (long*)malloc(sizeof(long) * (C + 1));
    C = 0;
    for (long p = 0; p < s->n; p++)
        if (cand[p]) ids[C++] = p;
    pair_hist* nh = NULL;
    long n_nh = 0, cap_nh = 0;
    double Jpq[3], un[3];
    if (brute) {
        for (long a = 0; a < C; a++)
            for (long b = a + 1; b < C; b++) {
                long p = ids[a], q = ids[b];
                if (excluded(s, p, q)) continue;
                if (pair_impulse(s, p, q, Jpq, un)) push_pair(&nh, &n_nh, &cap_nh, p, q, un, Jpq);
            }
    } else if (C > 0) {
        /* bin edge: every contacting pair has dist < R_p + R_q + dt |v_p - v_q| */
        double Rmax = 0.0, vmax = 0.0, lo[3] = {INFINITY, INFINITY, INFINITY};
        for (long a = 0; a < C; a++) {
            long p = ids[a];
            double R = radius(s, p), sp = norm3(&s->v[3 * p]);
            if (R > Rmax) Rmax = R;
            if (sp > vmax) vmax = sp;
            for (int j = 0; j < 3; j++)
                if (s->x[3 * p + j] < lo[j]) lo[j] = s->x[3 * p + j];
        }
        double h = 2.0 * Rmax + 2.0 * s->P.dt * vmax;
        if (!(h > 0.0)) h = s->P.dx;
        /* key = packed bin coordinates; sort (key, particle) pairs */
        long* kv = (long*)malloc(sizeof(long) * 2 * C);
        long dims[3] = {0, 0, 0};
        for (long a = 0; a < C; a++) {
            long p = ids[a];
            for (int j = 0; j < 3; j++) {
                long bj = (long)floor((s->x[3 * p + j] - lo[j]) / h);
                if (bj + 1 > dims[j]) dims[j] = bj + 1;
            }
        }
        for (long a = 0; a < C; a++) {
            long p = ids[a], b[3];
            for (int j = 0; j < 3; j++) b[j] = (long)floor((s->x[3 * p + j] - lo[j]) / h);
            kv[2 * a] = (b[2] * dims[1] + b[1]) * dims[0] + b[0];
            kv[2 * a + 1] = p;
        }
        qsort(kv, C, 2 * sizeof(long), cmp_long2);
        for (long a = 0; a < C; a++) {
            long p = kv[2 * a + 1], b[3];
            for (int j = 0; j < 3; j++) b[j] = (long)floor((s->x[3 * p + j] - lo[j]) / h);
            for (int dz = -1; dz <= 1; dz++)
                for (int dy = -1; dy <= 1; dy++)
                    for (int dx = -1; dx <= 1; dx++) {
                        long c0 = b[0] + dx, c1 = b[1] + dy, c2 = b[2] + dz;
                        if (c0 < 0 || c1 < 0 || c2 < 0 || c0 >= dims[0] || c1 >= dims[1] || c2 >= dims[2]) continue;
                        long key = (c2 * dims[1] + c1) * dims[0] + c0;
                        /* binary search for the first entry with this key */
                        long l = 0, r = C;
                        while (l < r) {
                            long m = (l + r) / 2;
                            if (kv[2 * m] < key)
                                l = m + 1;
                            else
                                r = m;
                        }
                        for (long i = l; i < C && kv[2 * i] == key; i++) {
                            long q = kv[2 * i + 1];
                            if (q <= p) continue;
                            if (excluded(s, p, q)) continue;
                            if (pair_impulse(s, p, q, Jpq, un)) push_pair(&nh, &n_nh, &cap_nh, p, q, un, Jpq);
                        }
                    }
        }
        free(kv);
    }
    /* deterministic application: pairs sorted by (p, q) */
    if (n_nh > 1) qsort(nh, n_nh, sizeof(pair_hist), cmp_pair);
    for (long i = 0; i < n_nh; i++) {
        long p = nh[i].p, q = nh[i].q;
        for (int j = 0; j < 3; j++) {
            s->J[3 * p + j] += nh[i].J[j];
            s->J[3 * q + j] -= nh[i].J[j];
        }
    }
    free(s->ph);
    s->ph = nh;
    s->n_ph = n_nh;
    s->cap_ph = cap_nh;
    s->last_pairs = n_nh;
    free(cand);
    free(ids);
}

/* ------------------------------------------------------------------------- */
/* Grid accumulators: one list per node, one entry per occupied code.          */
/* ------------------------------------------------------------------------- */
static node_entry* get_entry(orc_scene* s, long node, uint64_t code)
{
    node_entry** pp = &s->head[node];
    while (*pp && (*pp)->code < code) pp = &(*pp)->next;
    if (*pp && (*pp)->code == code) return *pp;
    if (s->n_pool == s->cap_pool) return NULL; /* pool sized for the worst case */
    node_entry* e = &s->pool[s->n_pool++];
    memset(e, 0, sizeof(*e));
    e->code = code;
    e->next = *pp;
    *pp = e;
    return e;
}

static node_entry* find_entry(orc_scene* s, long node, uint64_t code)
{
    for (node_entry* e = s->head[node]; e; e = e->next)
        if (e->code == code) return e;
    return NULL;
}

/* Couple all entries of one node for the field selected by which: 0 = (p, dp),
 * 1 = pt (MUSL re-scatter), following Eq. 8 and reading R6. */
static void couple_node(orc_scene* s, long node, int which)
{
    int S = 0;
    for (node_entry* e = s->head[node]; e; e = e->next) S++;
    if (S == 0) return;
    double* m = (double*)malloc(sizeof(double) * S);
    uint64_t* c = (uint64_t*)malloc(sizeof(uint64_t) * S);
    double* f = (double*)malloc(sizeof(double) * 3 * S);
    double* fb = (double*)malloc(sizeof(double) * 3 * S);
    int a = 0;
    for (node_entry* e = s->head[node]; e; e = e->next, a++) {
        m[a] = e->m;
        c[a] = e->code;
    }
    int K = s->P.max_cuts;
    for (int pass = 0; pass < (which == 0 ? 2 : 1); pass++) {
        a = 0;
        for (node_entry* e = s->head[node]; e; e = e->next, a++)
            for (int j = 0; j < 3; j++) f[3 * a + j] = which ? e->pt[j] : (pass ? e->dp[j] : e->p[j]);
        orc_couple(S, m, c, K, f, fb);
        a = 0;
        for (node_entry* e = s->head[node]; e; e = e->next, a++)
            for (int j = 0; j < 3; j++) {
                if (which)
                    e->ptbar[j] = fb[3 * a + j];
                else if (pass)
                    e->dpbar[j] = fb[3 * a + j];
                else
                    e->pbar[j] = fb[3 * a + j];
            }
    }
    free(m);
    free(c);
    free(f);
    free(fb);
}

/* ------------------------------------------------------------------------- */
/* One TLMPM substep (Sec. III-B to III-E, App.).                             */
/* wrench: [nt][6] force and torque per tool, the reaction of Eq. 16 summed    */
/* over particles for this substep (may be NULL).                              */
/* brute_pairs: 1 = all candidate pairs, 0 = binned search.                    */
/* Whole-rollout trajectories are "parity unpinned" beyond the invariants the  */
/* tests check (momentum balance, zero exchange, uniform translation, free     */
/* fall); two independent implementations agreeing is the remaining check.     */
/* ------------------------------------------------------------------------- */
int orc_step(orc_scene* s, const orc_tool* tools, int nt, double* wrench, int brute_pairs)
{
    const orc_params* P = &s->P;
    long n = s->n;
    double dt = P->dt;
    int K = P->max_cuts;
    if (nt < 0 || nt > ORC_MAX_RIGID - 1) return ORC_E_INVALID;
    s->status = ORC_OK;

    /* 1. contact impulses on x^n, v^n, c^n */
    memset(s->J, 0, sizeof(double) * 3 * n);
    if (wrench) memset(wrench, 0, sizeof(double) * 6 * nt);
    double* D_start = (double*)malloc(sizeof(double) * (n + 1));
    memcpy(D_start, s->D, sizeof(double) * n);
    if (P->floor_on) rigid_contact(s, 0, NULL, NULL, D_start);
    for (int t = 0; t < nt; t++)
        if (tools[t].contact) rigid_contact(s, 1 + t, &tools[t], wrench ? &wrench[6 * t] : NULL, D_start);
    free(D_start);
    if (P->material_contact)
        material_contact(s, brute_pairs);
    else
        s->n_ph = 0;

    /* 2. label-masked P2G (Eq. 2) with gravity and contact impulses */
    long nn = s->nodes[0] * s->nodes[1] * s->nodes[2];
    memset(s->head, 0, sizeof(node_entry*) * nn);
    const int ns = orc_stencil_nodes(P);
    if (s->cap_pool < ns * n + 8) {
        s->cap_pool = ns * n + 8;
        s->pool = (node_entry*)realloc(s->pool, sizeof(node_entry) * s->cap_pool);
    }
    s->n_pool = 0;
    long node[27];
    double w[27], g[81];
    /* first Piola-Kirchhoff stress of every particle at F^n (independent per particle) */
    double* Pall = (double*)malloc(sizeof(double) * 9 * (n + 1));
    int bad_any = 0;
#pragma omp parallel for reduction(| : bad_any)
    for (long p = 0; p < n; p++) {
        double* Pk = &Pall[9 * p];
        int bad;
        if (P->material == 1 && P->yield_stress > 0.0) {
            /* P = P_fcr(F_e) F_p^{-T}, F_e = F F_p^{-1} (reading R32) */
            double Fe[9], Pe[9];
            matmul3(&s->F[9 * p], &s->Fpi[9 * p], Fe);
            bad = orc_fcr_P(s->E[p], P->nu, Fe, Pe);
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) {
                    double a = 0.0;
                    for (int k = 0; k < 3; k++) a += Pe[3 * i + k] * s->Fpi[9 * p + 3 * j + k];
                    Pk[3 * i + j] = a;
                }
        } else {
            bad = P->material == 1 ? orc_fcr_P(s->E[p], P->nu, &s->F[9 * p], Pk)
                                   : orc_neo_hookean_P(s->E[p], P->nu, &s->F[9 * p], Pk);
        }
        if (bad) bad_any = 1;
        if (P->viscosity > 0.0) {
            double Pv[9];
            if (orc_visc_P(P->viscosity, &s->F[9 * p], &s->Fdot[9 * p], Pv)) bad_any = 1;
            for (int i = 0; i < 9; i++) Pk[i] += Pv[i];
        }
    }
    if (bad_any) s->status = ORC_E_NONFINITE;
    /* scatter into the node accumulators, serially in particle order */
    for (long p = 0; p < n; p++) {
        const double* Pk = &Pall[9 * p];
        orc_shape(P, &s->X[3 * p], node, w, g);
        uint64_t c = code_of(s, p);
        double mp = s->mass[p], V0 = s->vol0[p];
        double ext[3];
        for (int j = 0; j < 3; j++) ext[j] = s->J[3 * p + j] + dt * mp * P->gravity[j];
        for (int k = 0; k < ns; k++) {
            if (w[k] == 0.0) continue; /* reading R7: no contribution, no slot */
            node_entry* e = get_entry(s, node[k], c);
            e->m += w[k] * mp;
            for (int j = 0; j < 3; j++) {
                double PgN = Pk[3 * j + 0] * g[3 * k + 0] + Pk[3 * j + 1] * g[3 * k + 1] + Pk[3 * j + 2] * g[3 * k + 2];
                e->p[j] += w[k] * mp * s->v[3 * p + j];
                e->dp[j] += -dt * V0 * PgN + w[k] * ext[j];
            }
        }
    }

    free(Pall);

    /* 3. compatibility coupling (Eq. 8) */
#pragma omp parallel for schedule(dynamic, 4096)
    for (long i = 0; i < nn; i++) couple_node(s, i, 0);

    /* 4-5. grid update (Eq. 9) and PIC/FLIP G2P (Eq. 17); x moves with v^{n+1} (reading R4) */
    double* vnew = (double*)malloc(sizeof(double) * 3 * (n + 1));
#pragma omp parallel for
    for (long p = 0; p < n; p++) {
        long node[27];
        double w[27], g[81];
        orc_shape(P, &s->X[3 * p], node, w, g);
        uint64_t c = code_of(s, p);
        double acc_v[3] = {0, 0, 0}, acc_x[3] = {0, 0, 0};
        for (int k = 0; k < ns; k++) {
            if (w[k] == 0.0) continue;
            node_entry* e = find_entry(s, node[k], c);
            for (int j = 0; j < 3; j++) {
                double vn = e->pbar[j] / e->m;
                double dv = e->dpbar[j] / e->m;
                double vn1 = (e->pbar[j] + e->dpbar[j]) / e->m;
                acc_v[j] += w[k] * ((1.0 - P->beta) * vn + dv);
                acc_x[j] += w[k] * vn1;
            }
        }
        for (int j = 0; j < 3; j++) {
            vnew[3 * p + j] = P->beta * s->v[3 * p + j] + acc_v[j];
            s->x[3 * p + j] += dt * acc_x[j];
        }
    }
    memcpy(s->v, vnew, sizeof(double) * 3 * n);
    free(vnew);

    /* 6. MUSL re-scatter of m_p v_p^{n+1} with the same coupling */
    for (long p = 0; p < n; p++) {
        orc_shape(P, &s->X[3 * p], node, w, g);
        uint64_t c = code_of(s, p);
        for (int k = 0; k < ns; k++) {
            if (w[k] == 0.0) continue;
            node_entry* e = find_entry(s, node[k], c);
            for (int j = 0; j < 3; j++) e->pt[j] += w[k] * s->mass[p] * s->v[3 * p + j];
        }
    }
#pragma omp parallel for schedule(dynamic, 4096)
    for (long i = 0; i < nn; i++) couple_node(s, i, 1);
#pragma omp parallel for
    for (long k = 0; k < s->n_pool; k++) {
        node_entry* e = &s->pool[k];
        for (int j = 0; j < 3; j++) e->vt[j] = e->ptbar[j] / e->m;
    }

    /* 7. deformation gradient from the remapped velocities (reading R5) */
    int bad_F = 0;
#pragma omp parallel for reduction(| : bad_F)
    for (long p = 0; p < n; p++) {
        long node[27];
        double w[27], g[81];
        orc_shape(P, &s->X[3 * p], node, w, g);
        uint64_t c = code_of(s, p);
        double L[9] = {0};
        for (int k = 0; k < ns; k++) {
            if (w[k] == 0.0) continue;
            node_entry* e = find_entry(s, node[k], c);
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) L[3 * a + b] += e->vt[a] * g[3 * k + b];
        }
        double* F = &s->F[9 * p];
        for (int i = 0; i < 9; i++) F[i] += dt * L[i];
        memcpy(&s->Fdot[9 * p], L, sizeof(L));
        if (P->material == 1 && P->yield_stress > 0.0 && det3(F) > 0.0) {
            /* plasticity projection of the trial F_e = F F_p^{-1}; F_p^{-1} = F^{-1} F_e */
            double Fe[9], Fen[9], Fi[9];
            matmul3(F, &s->Fpi[9 * p], Fe);
            if (orc_vm_project(s->E[p], P->nu, P->yield_stress, Fe, Fen) == 1 && inv3(F, Fi) == 0)
                matmul3(Fi, Fen, &s->Fpi[9 * p]);
        }
        double J = det3(F);
        int finite = 1;
        for (int i = 0; i < 9; i++) finite &= isfinite(F[i]);
        if (!(J > 0.0) || !finite) bad_F = 1;
    }
    if (bad_F) s->status = ORC_E_NONFINITE;
    (void)K;
    return s->status;
}

/* ------------------------------------------------------------------------- */
/* Grid diagnostics of the last substep, for kernel-level comparisons.        */
/* Writes up to cap entries: node index, code, m, v^n = pbar/m,               */
/* v^{n+1} = (pbar+dpbar)/m and the remapped velocity vt.  Returns the count.  */
/* ------------------------------------------------------------------------- */
long orc_grid_dump(const orc_scene* s, long cap, int64_t* node_out, uint64_t* code_out, double* m_out,
                   double* vn_out, double* vn1_out, double* vt_out)
{
    long nn = s->nodes[0] * s->nodes[1] * s->nodes[2], k = 0;
    for (long i = 0; i < nn; i++)
        for (node_entry* e = s->head[i]; e; e = e->next) {
            if (k < cap) {
                node_out[k] = i;
                code_out[k] = e->code;
                m_out[k] = e->m;
                for (int j = 0; j < 3; j++) {
                    vn_out[3 * k + j] = e->pbar[j] / e->m;
                    vn1_out[3 * k + j] = (e->pbar[j] + e->dpbar[j]) / e->m;
                    vt_out[3 * k + j] = e->vt[j];
                }
            }
            k++;
        }
    return k;
}
