// tlmpm_device.h -- device functions shared by the trilinear (tlmpm_kernels.hip)
// and quadratic (tlmpm_quad.hip) transfer kernels and the contact kernels
// (tlmpm_contact.hip): side codes, the LDS barrier, the constitutive models and the
// slot-table pass (launched alone or beside the pair search).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "tlmpm_common.h"

#define DEV __device__ __forceinline__

// ---------------------------------------------------------------------------- codes
// A side code is held as two 15-bit masks: s1 has bit k set when digit k is 1, s2
// when it is 2 (Eq. 7 in another basis).  Two codes conflict iff some cut has side
// 1 in one and side 2 in the other (Sec. III-D).
DEV bool codes_conflict(uint32_t a, uint32_t b)
{
    uint32_t a1 = a & 0x7FFFu, a2 = (a >> 15) & 0x7FFFu;
    uint32_t b1 = b & 0x7FFFu, b2 = (b >> 15) & 0x7FFFu;
    return ((a1 & b2) | (a2 & b1)) != 0u;
}

DEV uint32_t slot_key(const SceneK& S, uint32_t code) { return S.single_field ? 0u : (code & TL_CODE_MASK); }

// ------------------------------------------------------------ displacement anchors
// Order-preserving map of a float to an unsigned key (larger float, larger key), so
// that a maximum over floats of either sign is an integer atomicMax; key 0 lies below
// the key of every float (the slots start at 0).
DEV uint32_t fkey(float f)
{
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

DEV float fkey_value(uint32_t k) { return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k); }

// Records the displacement anchor a and spread s of a brick (part 0) or of a split
// brick's later rounds (part 1): |u_p - a|_inf <= s for all its particles.  The
// scene bounds of a + s and s - a per axis go to the slot maxima of umm.
DEV void put_anchor(const SceneD& D, int bi, int brick, int part, const float a[3], float s)
{
    float* o = (part ? D.uanc_x : D.uanc) + (long long)brick * 4;
    o[0] = a[0];
    o[1] = a[1];
    o[2] = a[2];
    o[3] = s;
    uint32_t* mm = D.umm + (bi & (TL_USLOTS - 1));
    for (int k = 0; k < 3; k++) {
        atomicMax(mm + k * TL_USLOTS, fkey(a[k] + s));
        atomicMax(mm + (3 + k) * TL_USLOTS, fkey(s - a[k]));
    }
}

// Anchor of a G2P workgroup: the centre of a box record of the brick's particles
// after the last G2P (box) minus the centre of the box of their reference positions,
// the displacement of a rigid translation.  Any value serves (the spread is measured
// against it); this one follows the motion.
DEV void g2p_anchor(const SceneD& D, const float* box, int brick, float a[3])
{
    const float* rc = D.uref + (long long)brick * 4;
    for (int k = 0; k < 3; k++) a[k] = 0.5f * (box[k] + box[3 + k]) - rc[k];
}

// Current AABB and speed bound of an active brick: the box written by its G2P, joined
// with that of its second workgroup when the brick was split
DEV void brick_aabb(const SceneK& S, const SceneD& D, int bi, int brick, float bb[7])
{
    const float* a = D.aabb + (long long)brick * 8;
    if (S.xcap == 0) { // the scene never splits
#pragma unroll
        for (int q = 0; q < 7; q++) bb[q] = a[q];
        return;
    }
    // all loads issued together, then the join
    const float* x = D.aabb_x + (long long)brick * 8;
    float ra[7], rx[7];
#pragma unroll
    for (int q = 0; q < 7; q++) {
        ra[q] = a[q];
        rx[q] = x[q];
    }
    const bool join = D.xg[0] != 0 && D.xrs[bi] != 0;
#pragma unroll
    for (int q = 0; q < 7; q++) bb[q] = !join ? ra[q] : (q < 3 ? fminf(ra[q], rx[q]) : fmaxf(ra[q], rx[q]));
}

// Anchor a and spread s of all particles of active brick bi (= brick): the record of
// its last G2P, joined with that of the later rounds when that G2P split it.
DEV void brick_anchor(const SceneK& S, const SceneD& D, int bi, int brick, float a[3], float& s)
{
    const float* r = D.uanc + (long long)brick * 4;
    a[0] = r[0];
    a[1] = r[1];
    a[2] = r[2];
    s = r[3];
    if (S.xcap > 0 && D.xg[0] != 0 && D.xrs[bi] != 0) {
        const float* x = D.uanc_x + (long long)brick * 4;
        float t = 0.0f;
        for (int k = 0; k < 3; k++) t = fmaxf(t, fabsf(x[k] - a[k]));
        s = fmaxf(s, x[3] + t);
    }
}

// Workgroup barrier that orders LDS only: global loads issued before it stay in
// flight (a full __syncthreads() would also wait for them).
DEV void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ------------------------------------------------------------- constitutive model
// Compressible Neo-Hookean first Piola-Kirchhoff stress written in H = F - I so
// that small strains keep their relative precision in FP32:
//   cof(F) = (1 + tr H) I - H^T + cof(H),  J = 1 + tr H + I2(H) + det H,
//   F - F^{-T} = [(I2 + det H) I + J H + H^T - cof(H)] / J,
//   P = mu (F - F^{-T}) + lambda ln J F^{-T}.
// Returns false when J <= 0 or the state is not finite.
DEV bool neo_hookean(float E, float nu, const float* H, float* P)
{
    const float mu = E / (2.0f * (1.0f + nu));
    const float lam = E * nu / ((1.0f + nu) * (1.0f - 2.0f * nu));
    float cH[9];
    cH[0] = H[4] * H[8] - H[5] * H[7];
    cH[1] = H[5] * H[6] - H[3] * H[8];
    cH[2] = H[3] * H[7] - H[4] * H[6];
    cH[3] = H[2] * H[7] - H[1] * H[8];
    cH[4] = H[0] * H[8] - H[2] * H[6];
    cH[5] = H[1] * H[6] - H[0] * H[7];
    cH[6] = H[1] * H[5] - H[2] * H[4];
    cH[7] = H[2] * H[3] - H[0] * H[5];
    cH[8] = H[0] * H[4] - H[1] * H[3];
    const float trH = H[0] + H[4] + H[8];
    const float I2 = cH[0] + cH[4] + cH[8];
    const float I3 = H[0] * cH[0] + H[1] * cH[1] + H[2] * cH[2];
    const float Jm1 = trH + (I2 + I3);
    const float J = 1.0f + Jm1;
    if (!(J > 0.0f) || !isfinite(J)) return false;
    const float invJ = 1.0f / J;
    const float lnJ = log1pf(Jm1);
    const float e0 = I2 + I3;
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int s = 0; s < 3; s++) {
            int rs = 3 * r + s, sr = 3 * s + r;
            float id = (r == s) ? 1.0f : 0.0f;
            float FmFiT = (id * e0 + J * H[rs] + H[sr] - cH[rs]) * invJ;
            float FiT = (id * (1.0f + trH) - H[sr] + cH[rs]) * invJ;
            P[rs] = mu * FmFiT + lam * lnJ * FiT;
        }
    return true;
}

// Fixed-corotated first Piola-Kirchhoff stress P = 2 mu (F - R) + lambda (J - 1)
// J F^{-T} (Sec. III-B), F = R S the polar decomposition, in terms of H = F - I so
// that small strains keep their precision in FP32: with E = F^T F - I = H + H^T +
// H^T H = Q diag(e) Q^T (Jacobi rotations), S - I = Q diag(e / (sqrt(1 + e) + 1)) Q^T,
// S^{-1} = Q diag(1 / sqrt(1 + e)) Q^T, R = F S^{-1} and F - R = R (S - I).
// Returns false when J <= 0 or the state is not finite.
DEV bool fixed_corotated(float E, float nu, const float* H, float* P)
{
    const float mu = E / (2.0f * (1.0f + nu));
    const float lam = E * nu / ((1.0f + nu) * (1.0f - 2.0f * nu));
    float A[9];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            float a = H[3 * i + j] + H[3 * j + i];
#pragma unroll
            for (int k = 0; k < 3; k++) a += H[3 * k + i] * H[3 * k + j];
            A[3 * i + j] = a;
        }
    float Q[9] = {1.0f, 0.0f, 0.0f, 0.0f, 1.0f, 0.0f, 0.0f, 0.0f, 1.0f};
    // cyclic Jacobi sweeps (a fixed count: FP32 converges within four)
#pragma unroll 1
    for (int sweep = 0; sweep < 4; sweep++) {
#pragma unroll
        for (int pq = 0; pq < 3; pq++) {
            const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
            const float apq = A[3 * p + q];
            if (apq == 0.0f) continue;
            const float th = (A[3 * q + q] - A[3 * p + p]) / (2.0f * apq);
            const float t = copysignf(1.0f, th) / (fabsf(th) + sqrtf(th * th + 1.0f));
            const float c = 1.0f / sqrtf(t * t + 1.0f), sn = t * c;
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const float akp = A[3 * k + p], akq = A[3 * k + q];
                A[3 * k + p] = c * akp - sn * akq;
                A[3 * k + q] = sn * akp + c * akq;
            }
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const float apk = A[3 * p + k], aqk = A[3 * q + k];
                A[3 * p + k] = c * apk - sn * aqk;
                A[3 * q + k] = sn * apk + c * aqk;
            }
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const float qkp = Q[3 * k + p], qkq = Q[3 * k + q];
                Q[3 * k + p] = c * qkp - sn * qkq;
                Q[3 * k + q] = sn * qkp + c * qkq;
            }
        }
    }
    float sm1[3], sinv[3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const float e = A[4 * k], r = sqrtf(1.0f + e);
        if (!(1.0f + e > 0.0f)) return false;
        sm1[k] = e / (r + 1.0f);
        sinv[k] = 1.0f / r;
    }
    float SmI[9], Si[9];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            float a = 0.0f, b = 0.0f;
#pragma unroll
            for (int k = 0; k < 3; k++) {
                a += Q[3 * i + k] * sm1[k] * Q[3 * j + k];
                b += Q[3 * i + k] * sinv[k] * Q[3 * j + k];
            }
            SmI[3 * i + j] = a;
            Si[3 * i + j] = b;
        }
    float Rm[9];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            float a = Si[3 * i + j];
#pragma unroll
            for (int k = 0; k < 3; k++) a += H[3 * i + k] * Si[3 * k + j];
            Rm[3 * i + j] = a;
        }
    float cH[9];
    cH[0] = H[4] * H[8] - H[5] * H[7];
    cH[1] = H[5] * H[6] - H[3] * H[8];
    cH[2] = H[3] * H[7] - H[4] * H[6];
    cH[3] = H[2] * H[7] - H[1] * H[8];
    cH[4] = H[0] * H[8] - H[2] * H[6];
    cH[5] = H[1] * H[6] - H[0] * H[7];
    cH[6] = H[1] * H[5] - H[2] * H[4];
    cH[7] = H[2] * H[3] - H[0] * H[5];
    cH[8] = H[0] * H[4] - H[1] * H[3];
    const float trH = H[0] + H[4] + H[8];
    const float I2 = cH[0] + cH[4] + cH[8];
    const float I3 = H[0] * cH[0] + H[1] * cH[1] + H[2] * cH[2];
    const float Jm1 = trH + (I2 + I3);
    if (!(1.0f + Jm1 > 0.0f) || !isfinite(Jm1)) return false;
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            float fr = 0.0f; // (F - R)_rc = (R (S - I))_rc
#pragma unroll
            for (int k = 0; k < 3; k++) fr += Rm[3 * r + k] * SmI[3 * k + c];
            const float cof = (r == c ? 1.0f + trH : 0.0f) - H[3 * c + r] + cH[3 * r + c]; // J F^{-T}
            P[3 * r + c] = 2.0f * mu * fr + lam * Jm1 * cof;
        }
    return true;
}

// Adds the Newtonian viscous first Piola-Kirchhoff stress J eta (l + l^T) F^{-T},
// l = Fdot F^{-1} (Sec. III-B), to P.  F = I + H with J > 0.
DEV void add_viscous(float eta, const float* H, const float* Fdot, float* P)
{
    float C[9]; // J F^{-T}
    C[0] = (1.0f + H[4]) * (1.0f + H[8]) - H[5] * H[7];
    C[1] = H[5] * H[6] - H[3] * (1.0f + H[8]);
    C[2] = H[3] * H[7] - (1.0f + H[4]) * H[6];
    C[3] = H[2] * H[7] - H[1] * (1.0f + H[8]);
    C[4] = (1.0f + H[0]) * (1.0f + H[8]) - H[2] * H[6];
    C[5] = H[1] * H[6] - (1.0f + H[0]) * H[7];
    C[6] = H[1] * H[5] - H[2] * (1.0f + H[4]);
    C[7] = H[2] * H[3] - (1.0f + H[0]) * H[5];
    C[8] = (1.0f + H[0]) * (1.0f + H[4]) - H[1] * H[3];
    const float J = (1.0f + H[0]) * C[0] + H[1] * C[1] + H[2] * C[2];
    const float iJ = 1.0f / J;
    float l[9]; // Fdot F^{-1}, F^{-1} = C^T / J
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            float a = 0.0f;
#pragma unroll
            for (int k = 0; k < 3; k++) a += Fdot[3 * i + k] * C[3 * j + k];
            l[3 * i + j] = a * iJ;
        }
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            float a = 0.0f;
#pragma unroll
            for (int k = 0; k < 3; k++) a += eta * (l[3 * i + k] + l[3 * k + i]) * C[3 * k + j];
            P[3 * i + j] += a;
        }
}

// von Mises plasticity projection (Sec. III-B; reading R32) of the trial elastic
// deformation gradient F_e = F F_p^{-1} = I + K: with F_e^T F_e - I = K + K^T +
// K^T K = V diag(e) V^T, Hencky strain eps = log1p(e) / 2, the deviatoric part is
// scaled back onto |2 mu dev(eps)| = sqrt(2/3) sigma_y (volume kept).  The
// projected F_e = F_e M with M = V diag(exp(eps_new - eps)) V^T, so F_p^{-1} = I +
// G becomes (I + G) M.  Updates G and K; returns whether it yielded.
DEV bool vm_project(float E, float nu, float sigma_y, float* K, float* G)
{
    const float mu = E / (2.0f * (1.0f + nu));
    float A[9];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            float a = K[3 * i + j] + K[3 * j + i];
#pragma unroll
            for (int k = 0; k < 3; k++) a += K[3 * k + i] * K[3 * k + j];
            A[3 * i + j] = a;
        }
    float V[9] = {1.0f, 0.0f, 0.0f, 0.0f, 1.0f, 0.0f, 0.0f, 0.0f, 1.0f};
#pragma unroll 1
    for (int sweep = 0; sweep < 4; sweep++) {
#pragma unroll
        for (int pq = 0; pq < 3; pq++) {
            const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
            const float apq = A[3 * p + q];
            if (apq == 0.0f) continue;
            const float th = (A[3 * q + q] - A[3 * p + p]) / (2.0f * apq);
            const float t = copysignf(1.0f, th) / (fabsf(th) + sqrtf(th * th + 1.0f));
            const float c = 1.0f / sqrtf(t * t + 1.0f), sn = t * c;
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const float akp = A[3 * k + p], akq = A[3 * k + q];
                A[3 * k + p] = c * akp - sn * akq;
                A[3 * k + q] = sn * akp + c * akq;
            }
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const float apk = A[3 * p + k], aqk = A[3 * q + k];
                A[3 * p + k] = c * apk - sn * aqk;
                A[3 * q + k] = sn * apk + c * aqk;
            }
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const float vkp = V[3 * k + p], vkq = V[3 * k + q];
                V[3 * k + p] = c * vkp - sn * vkq;
                V[3 * k + q] = sn * vkp + c * vkq;
            }
        }
    }
    float eps[3];
#pragma unroll
    for (int k = 0; k < 3; k++) eps[k] = 0.5f * log1pf(A[4 * k]);
    const float tr = (eps[0] + eps[1] + eps[2]) * (1.0f / 3.0f);
    float dev[3], nd = 0.0f;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        dev[k] = eps[k] - tr;
        nd += dev[k] * dev[k];
    }
    nd = sqrtf(nd);
    const float lim = 0.816496580927726f * sigma_y; // sqrt(2/3)
    if (!(2.0f * mu * nd > lim)) return false;
    const float scale = lim / (2.0f * mu * nd);
    float d[3];
#pragma unroll
    for (int k = 0; k < 3; k++) d[k] = expm1f((scale - 1.0f) * dev[k]);
    float Mm[9]; // M - I
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) Mm[3 * i + j] = V[3 * i] * d[0] * V[3 * j] + V[3 * i + 1] * d[1] * V[3 * j + 1] +
                                                    V[3 * i + 2] * d[2] * V[3 * j + 2];
    float Gn[9], Kn[9];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            float g = G[3 * i + j] + Mm[3 * i + j], k = K[3 * i + j] + Mm[3 * i + j];
#pragma unroll
            for (int m = 0; m < 3; m++) {
                g += G[3 * i + m] * Mm[3 * m + j];
                k += K[3 * i + m] * Mm[3 * m + j];
            }
            Gn[3 * i + j] = g;
            Kn[3 * i + j] = k;
        }
#pragma unroll
    for (int a = 0; a < 9; a++) {
        G[a] = Gn[a];
        K[a] = Kn[a];
    }
    return true;
}

// ------------------------------------------------------------------- slot tables
// For every node: the distinct codes of the particles in its 8 incident cells, in
// ascending order (compact slots, Sec. III-G).  Skipped (count copied) when the
// labels did not change since the source table was built.
DEV void slots_body(const SceneK& S, const SceneD& D, int bi, int dst, int src, int force)
{
    const long long id = (long long)bi * blockDim.x + threadIdx.x;
    if (id >= S.NN) return;
    long long nb = id >> 6;
    int lid = (int)(id & 63);
    int hx = (int)(nb % S.nbx), hy = (int)((nb / S.nbx) % S.nby), hz = (int)(nb / ((long long)S.nbx * S.nby));
    bool rebuild = force != 0;
    const int stamp = D.ctr[0];
    if (!rebuild) {
        // a node depends on the cells of bricks h - {0,1}^3
        int any = 0;
#pragma unroll
        for (int d = 0; d < 8; d++) {
            int bx = hx - (d & 1), by = hy - ((d >> 1) & 1), bz = hz - ((d >> 2) & 1);
            if (bx < 0 || by < 0 || bz < 0 || bx >= S.cbx || by >= S.cby || bz >= S.cbz) continue;
            any |= D.bdirty[((long long)bz * S.cby + by) * S.cbx + bx] == stamp;
        }
        rebuild = any != 0;
    }
    if (!rebuild) {
        if (dst != src) {
            int c = D.cnt[src][id];
            D.cnt[dst][id] = (uint8_t)c;
            for (int s = 0; s < c; s++) D.scode[dst][s * S.NN + id] = D.scode[src][s * S.NN + id];
        }
        return;
    }
    int gx = hx * 4 + (lid & 3), gy = hy * 4 + ((lid >> 2) & 3), gz = hz * 4 + (lid >> 4);
    uint32_t codes[TL_SCAP_MAX];
    int c = 0;
    bool over = false;
    auto insert = [&](uint32_t k) {
        int pos = 0;
        while (pos < c && codes[pos] < k) pos++;
        if (pos < c && codes[pos] == k) return;
        if (c == S.scap) {
            over = true;
            return;
        }
        for (int q = c; q > pos; q--) codes[q] = codes[q - 1];
        codes[pos] = k;
        c++;
    };
    if (gx <= S.cx && gy <= S.cy && gz <= S.cz) {
        // the 8 incident cells: their one-key summaries, all loaded before use
        long long cell[8];
        uint32_t cc[8];
#pragma unroll
        for (int d = 0; d < 8; d++) {
            int x = gx - (d & 1), y = gy - ((d >> 1) & 1), z = gz - ((d >> 2) & 1);
            cell[d] = -1;
            cc[d] = TL_CC_EMPTY;
            if (x < 0 || y < 0 || z < 0 || x >= S.cx || y >= S.cy || z >= S.cz) continue;
            long long brick = ((long long)(z >> 2) * S.cby + (y >> 2)) * S.cbx + (x >> 2);
            int lx = x & 3, ly = y & 3, lz = z & 3;
            int w = (lx & 1) | ((ly & 1) << 1) | ((lz & 1) << 2);
            int i = (lx >> 1) | ((ly >> 1) << 1) | ((lz >> 1) << 2);
            cell[d] = brick * TL_CELLS + w * 8 + i;
            cc[d] = D.ccode[cell[d]];
        }
        for (int d = 0; d < 8; d++) {
            if (cc[d] == TL_CC_EMPTY) continue;
            if (cc[d] < TL_CC_FEW) {
                insert(cc[d]);
            } else if (cc[d] != TL_CC_MIXED) {
                const int n = (int)(cc[d] & 7u);
                uint32_t kk[TL_CKEYS];
#pragma unroll
                for (int k = 0; k < TL_CKEYS; k++) kk[k] = k < n ? D.ckeys[cell[d] * TL_CKEYS + k] : 0u;
#pragma unroll
                for (int k = 0; k < TL_CKEYS; k++)
                    if (k < n) insert(kk[k]);
            } else {
                for (int p = D.cell_start[cell[d]]; p < D.cell_start[cell[d] + 1]; p++) insert(slot_key(S, D.code[p]));
            }
        }
    }
    if (over) atomicOr(D.status, TL_ST_SLOT);
    D.cnt[dst][id] = (uint8_t)c;
    for (int s = 0; s < c; s++) D.scode[dst][s * S.NN + id] = codes[s];
}
