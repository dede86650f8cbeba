// tlmpm_reach.h -- reach tests that let contact work skip what cannot touch
// (Sec. III-E): can a tool's blade rectangle touch any particle of a brick during
// this substep (Eqs. 14-16), and can a material-contact candidate have a partner at
// all (Eqs. 10-13 with the reference-neighbour exclusion)?  Host and device code, so
// that both can be checked on the CPU.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "tlmpm_common.h"

// A particle at x with radius R <= Rmax and speed |v| <= vmax takes an impulse from
// tool T only when its predicted gap is negative (Eq. 14):
//   |x - x_c| - R + dt min((v - v_B(x_c)).n_B, 0) < 0,
// x_c its closest point on the rectangle, v_B(x_c) = v_B + w_B x (x_c - x_B).  Hence
//   |x - x_c| < Rmax + dt (vmax + |v_B| + |w_B| |x_c - x_B|),
// and |x_c - x_B| <= |x_e - x_B| + half_len + b_back since x_c = x_e + a e - b d with
// |a| <= half_len, 0 <= b <= b_back.  The distance to the rectangle is at least the
// gap between the projections of x and of the rectangle on any axis; the test takes
// the grid axes (the rectangle's bounding box) and the blade axes n, e, d, on which
// the rectangle spans s = 0, l in [-half_len, half_len], f in [-b_back, 0] about
// x_e.  bb[0..2] / bb[3..5]: smallest / largest FP32 current coordinate over the
// brick's particles, bb[6]: largest |v|.  The 1e-5 m of slack covers the FP32
// rounding of the box (half an ulp of a coordinate) and of the FP32 contact
// arithmetic.  jdt: time of the substep within the call, for tools whose pose
// advances with their velocity (TL_TOOL_ADVANCE), as in the contact itself.
// False means no particle of the brick can be touched; true may still find none.
__host__ __device__ inline bool brick_near_tool(const float* bb, const DevTool& T, float Rmax, float dt, double jdt)
{
    const DevBlade& B = T.b;
    const double adv = (T.flags & TL_TOOL_ADVANCE) ? jdt : 0.0;
    double xe[3], arm2 = 0.0, vb2 = 0.0, w2 = 0.0;
    for (int a = 0; a < 3; a++) {
        xe[a] = B.xe[a] + adv * B.ve[a];
        const double o = xe[a] - (T.xB[a] + adv * T.vB[a]);
        arm2 += o * o;
        vb2 += T.vB[a] * T.vB[a];
        w2 += (double)T.wB[a] * (double)T.wB[a];
    }
    const double vtool = sqrt(vb2) + sqrt(w2) * (sqrt(arm2) + B.half_len + B.b_back);
    const double reach = (double)Rmax + (double)dt * ((double)bb[6] + vtool) + 1e-5;
    double c[3], h[3];
    for (int a = 0; a < 3; a++) {
        // grid axis a: the rectangle spans x_e +- half_len |e_a| plus the back extent along -d
        const double back = -B.b_back * B.d[a];
        const double lo = xe[a] - B.half_len * fabs(B.e[a]) + fmin(back, 0.0);
        const double hi = xe[a] + B.half_len * fabs(B.e[a]) + fmax(back, 0.0);
        if ((double)bb[a] > hi + reach || (double)bb[3 + a] < lo - reach) return false;
        c[a] = 0.5 * ((double)bb[a] + (double)bb[3 + a]) - xe[a];
        h[a] = 0.5 * ((double)bb[3 + a] - (double)bb[a]);
    }
    const double* axis[3] = {B.n, B.e, B.d};
    const double ilo[3] = {0.0, -B.half_len, -B.b_back}, ihi[3] = {0.0, B.half_len, 0.0};
    for (int k = 0; k < 3; k++) {
        const double* q = axis[k];
        const double pc = c[0] * q[0] + c[1] * q[1] + c[2] * q[2];
        const double r = h[0] * fabs(q[0]) + h[1] * fabs(q[1]) + h[2] * fabs(q[2]);
        if (pc - r > ihi[k] + reach || pc + r < ilo[k] - reach) return false;
    }
    return true;
}

// The floor (plane z = floor_z, normal +z, at rest): a particle takes an impulse only
// when z - R + dt min(v_z, 0) < floor_z, so z < floor_z + Rmax + dt vmax.
__host__ __device__ inline bool brick_near_floor(const float* bb, float floor_z, float Rmax, float dt)
{
    return bb[2] - Rmax - dt * bb[6] - 1e-6f <= floor_z;
}

// Material contact: a candidate p (reference brick b) is searched for partners q
// within the bin edge hb in the current configuration, |x_p - x_q| < hb; a pair of
// reference neighbours (reference cells at most one apart per axis) with compatible
// side codes is excluded.  With x = X + u, per axis |X_p - X_q| <= |x_p - x_q| +
// |u_p - u_q|.  U[k]: the range of the displacements of the whole scene along axis
// k; Dk[k]: a bound on |u_p - u_q| along k for p in b and q in the 27 bricks around
// it (b included).  True when
//  - no particle of a brick outside the 27 can be within hb: such a brick's
//    reference positions are more than 4 dx from p's along some axis, so it needs
//    U[k] > 4 dx - hb along that axis;
//  - every particle of the 27 bricks within hb is a reference neighbour of p:
//    |X_p - X_q| < hb + Dk[k] <= dx along every axis.
// Then p can only have a partner whose side code conflicts with its own.  M bounds
// the magnitude of the coordinates: the slack covers the FP32 rounding of x =
// fl(X + u) (half an ulp of each coordinate), of the reach test and of the bounds'
// own arithmetic (a relative 1e-5 on U and Dk).
__host__ __device__ inline bool pair_skip_bounds_ok(const float U[3], const float Dk[3], float hb, float dx, float M)
{
    const float slack = 4e-7f * (M + hb) + 1e-6f * dx;
    for (int k = 0; k < 3; k++) {
        if (!(U[k] * (1.0f + 1e-5f) + hb + slack <= 4.0f * dx)) return false;
        if (!(Dk[k] * (1.0f + 1e-5f) + hb + slack <= dx)) return false;
    }
    return true;
}
