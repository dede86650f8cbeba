// tlmpm_band.h -- the blade band of a cut (Sec. III-C, Eqs. 3, 4, 6): the side
// digit one blade assigns to one particle, and the test that lets the label pass
// skip a whole brick.  Host and device functions, so that the skip test can be
// checked exhaustively on the CPU.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "tlmpm_common.h"

// Side digit of a particle at x with velocity v for blade B (0: not assigned):
//   r = x - x_e;  s = r.n, l = r.e, f = r.d  (Eq. 3), u_c = (v_e - v).d;
//   in the band iff |s| <= h, |l| <= L, -b_back - max(u_c dt, 0) <= f <= b_lead (Eq. 4);
//   assigned iff in the band and f <= 0: 1 if s < 0, else 2 (Eq. 6, s = 0 -> 2).
// FP64 with the sums in a fixed order and no contraction, the order the CPU
// reference uses, so that both sides decide identically from the same FP32 state.
__host__ __device__ inline int label_digit(const double x[3], const double v[3], const DevBlade& B, double dt)
{
#pragma clang fp contract(off)
    double r0 = x[0] - B.xe[0], r1 = x[1] - B.xe[1], r2 = x[2] - B.xe[2];
    double s = (r0 * B.n[0] + r1 * B.n[1]) + r2 * B.n[2];
    double l = (r0 * B.e[0] + r1 * B.e[1]) + r2 * B.e[2];
    double f = (r0 * B.d[0] + r1 * B.d[1]) + r2 * B.d[2];
    double uc = ((B.ve[0] - v[0]) * B.d[0] + (B.ve[1] - v[1]) * B.d[1]) + (B.ve[2] - v[2]) * B.d[2];
    double lo = -B.b_back - fmax(uc * dt, 0.0);
    bool in_band = fabs(s) <= B.half_width && fabs(l) <= B.half_len && lo <= f && f <= B.b_lead;
    if (!in_band || !(f <= 0.0)) return 0;
    return (s < 0.0) ? 1 : 2;
}

// Can blade B assign a digit to any particle of a brick whose box is bb?
// bb[0..2] / bb[3..5]: smallest / largest FP32 current coordinate fl(X + u) over the
// brick's particles, bb[6]: largest |v|.  label_digit sees the exact X + u (FP64),
// which can lie half an FP32 ulp outside fl(X + u); the box is therefore first
// widened by one ulp outward on every face (nextafterf), which contains every exact
// position whatever the rounding.  The band extents get a further 1e-9 m for the
// FP64 rounding of the projections.  False means no particle of the brick is in
// the band (conservative: true may still find none).
__host__ __device__ inline bool brick_near_band(const float* bb, const DevBlade& B, double dt)
{
    double lo3[3], hi3[3];
    for (int a = 0; a < 3; a++) {
        lo3[a] = (double)nextafterf(bb[a], -INFINITY);
        hi3[a] = (double)nextafterf(bb[3 + a], INFINITY);
    }
    // band extents in (s, l, f); the rear bound grows by max(u_c dt, 0) <= (|v_e| + max |v|) dt
    double ucmax = sqrt(B.ve[0] * B.ve[0] + B.ve[1] * B.ve[1] + B.ve[2] * B.ve[2]) + (double)bb[6];
    double flo = -B.b_back - ucmax * dt - 1e-9, fhi = B.b_lead + 1e-9;
    double smin = 1e300, smax = -1e300, lmin = 1e300, lmax = -1e300, fmn = 1e300, fmx = -1e300;
    for (int c = 0; c < 8; c++) {
        double pt[3] = {(c & 1) ? hi3[0] : lo3[0], (c & 2) ? hi3[1] : lo3[1], (c & 4) ? hi3[2] : lo3[2]};
        double r[3] = {pt[0] - B.xe[0], pt[1] - B.xe[1], pt[2] - B.xe[2]};
        double s = r[0] * B.n[0] + r[1] * B.n[1] + r[2] * B.n[2];
        double l = r[0] * B.e[0] + r[1] * B.e[1] + r[2] * B.e[2];
        double f = r[0] * B.d[0] + r[1] * B.d[1] + r[2] * B.d[2];
        smin = fmin(smin, s);
        smax = fmax(smax, s);
        lmin = fmin(lmin, l);
        lmax = fmax(lmax, l);
        fmn = fmin(fmn, f);
        fmx = fmax(fmx, f);
    }
    double h = B.half_width + 1e-9, L = B.half_len + 1e-9;
    return !(smin > h || smax < -h || lmin > L || lmax < -L || fmn > fhi || fmx < flo);
}
