// Host-side check of rigid contact's brick skip test (tlmpm_reach.h): a brick whose
// particle takes a tool impulse must never be skipped.  Random blade rectangles in
// random orientations, moving and spinning (free tools), some with poses advanced
// within the call; particles placed about a random point of the rectangle (face,
// edge or corner), at distances around the contact reach.  The contact predicate is
// evaluated here from its definition in FP64: closest point of the rectangle,
// n_B = (x - x_c) / |x - x_c|, v_B(x_c) = v_B + w_B x (x_c - x_B), contact iff
// |x - x_c| - R + dt min((v - v_B(x_c)).n_B, 0) < 0 (Eq. 14).
// Prints "cases <n> contact <k> missed <m> norot_missed <r> pruned <p>":
// m (must be 0) counts contacts whose brick the test skips, r the contacts that the
// same reach without the tool's spin term would skip, p the non-contact bricks that
// pass the rectangle's bounding-box test but fail a blade-axis test.
// Runs on the CPU only (no HIP runtime call).
#include <math.h>
#include <stdint.h>
#include <stdio.h>

#include "../../paper_2609_27342_amd/csrc/tlmpm_reach.h"

static uint64_t g_state = 0x2545F4914F6CDD1Dull;
static double urand()
{
    g_state ^= g_state << 13;
    g_state ^= g_state >> 7;
    g_state ^= g_state << 17;
    return (double)(g_state >> 11) * (1.0 / 9007199254740992.0);
}

static void unit(double* a)
{
    double n = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    for (int i = 0; i < 3; i++) a[i] /= n;
}

static void cross(const double* a, const double* b, double* c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// the rectangle's bounding box alone, with the given reach (the grid-axis part)
static bool bbox_only(const float* bb, const DevTool& T, double reach, double jdt)
{
    const DevBlade& B = T.b;
    const double adv = (T.flags & TL_TOOL_ADVANCE) ? jdt : 0.0;
    for (int a = 0; a < 3; a++) {
        double lo = 1e30, hi = -1e30;
        for (int c = 0; c < 4; c++) {
            double al = (c & 1) ? B.half_len : -B.half_len, be = (c & 2) ? B.b_back : 0.0;
            double p = B.xe[a] + adv * B.ve[a] + al * B.e[a] - be * B.d[a];
            lo = fmin(lo, p);
            hi = fmax(hi, p);
        }
        if (bb[a] > hi + reach || bb[3 + a] < lo - reach) return false;
    }
    return true;
}

int main()
{
    long cases = 0, contact = 0, missed = 0, norot_missed = 0, pruned = 0;
    for (int trial = 0; trial < 300000; trial++) {
        const float dt = (trial & 1) ? 1e-4f : 3e-5f;
        double n[3], d[3], e[3];
        if (trial % 5 == 0) { // axis-aligned blade
            int ax = (trial / 5) % 3;
            n[0] = n[1] = n[2] = 0.0;
            n[ax] = 1.0;
            d[0] = d[1] = d[2] = 0.0;
            d[(ax + 1) % 3] = -1.0;
        } else {
            double r[3] = {urand() - 0.5, urand() - 0.5, urand() - 0.5}, t[3] = {urand() - 0.5, urand() - 0.5, urand() - 0.5};
            unit(r);
            double k = dot(t, r);
            for (int i = 0; i < 3; i++) t[i] -= k * r[i];
            unit(t);
            for (int i = 0; i < 3; i++) {
                n[i] = r[i];
                d[i] = t[i];
            }
        }
        cross(n, d, e);
        DevTool T = {};
        DevBlade& B = T.b;
        B.half_len = 0.02 + 0.1 * urand();
        B.half_width = 0.01;
        B.b_back = 0.01 + 0.05 * urand();
        B.b_lead = 0.002;
        for (int i = 0; i < 3; i++) {
            B.n[i] = n[i];
            B.d[i] = d[i];
            B.e[i] = e[i];
            B.xe[i] = 0.05 + 0.2 * urand();
            B.ve[i] = (urand() - 0.5) * 2.0;
            T.vB[i] = B.ve[i];
            T.xB[i] = B.xe[i] + (urand() - 0.5) * 0.1; // centre of mass off the edge
            T.wB[i] = (float)((trial % 3 == 0) ? 0.0 : (urand() - 0.5) * 200.0);
        }
        T.flags = TL_TOOL_CONTACT | ((trial % 4 == 1) ? TL_TOOL_ADVANCE : 0u);
        const double jdt = (trial % 4 == 1) ? 7.0 * dt : 0.0;
        const double adv = (T.flags & TL_TOOL_ADVANCE) ? jdt : 0.0;
        double xe[3], xB[3];
        for (int i = 0; i < 3; i++) {
            xe[i] = B.xe[i] + adv * B.ve[i];
            xB[i] = T.xB[i] + adv * T.vB[i];
        }
        const float Rmax = 0.0004f + 0.0008f * (float)urand();
        const double R = Rmax * (0.5 + 0.5 * urand());
        // a point of the rectangle: interior, on an edge or at a corner
        double al = (2.0 * urand() - 1.0) * B.half_len, be = urand() * B.b_back;
        const int where = trial % 7;
        if (where == 1 || where == 3) al = (al < 0 ? -1.0 : 1.0) * B.half_len;
        if (where == 2 || where == 3) be = (urand() < 0.5) ? 0.0 : B.b_back;
        double xc0[3];
        for (int i = 0; i < 3; i++) xc0[i] = xe[i] + al * e[i] - be * d[i];
        // the particle: a random direction away from that point, at a distance around the reach
        double dir[3] = {urand() - 0.5, urand() - 0.5, urand() - 0.5};
        unit(dir);
        double v[3];
        const double vmax_p = 2.0 * urand();
        double vd[3] = {urand() - 0.5, urand() - 0.5, urand() - 0.5};
        unit(vd);
        for (int i = 0; i < 3; i++) v[i] = vmax_p * vd[i];
        const double wn = sqrt((double)T.wB[0] * T.wB[0] + (double)T.wB[1] * T.wB[1] + (double)T.wB[2] * T.wB[2]);
        const double scale = R + dt * (vmax_p + 2.0 + wn * 0.2);
        double dist0 = urand() * 1.5 * scale;
        if (trial % 11 == 10) { // well off the plane, inside the rectangle's bounding box when it is oblique
            for (int i = 0; i < 3; i++) dir[i] = (trial & 2) ? n[i] : -n[i];
            dist0 = scale + 0.008 + 0.02 * urand();
        }
        double x[3];
        for (int i = 0; i < 3; i++) x[i] = xc0[i] + dist0 * dir[i];
        cases++;
        // exact contact predicate: closest point by clamping in the blade frame
        double r[3] = {x[0] - xe[0], x[1] - xe[1], x[2] - xe[2]};
        double a = fmin(fmax(dot(r, e), -B.half_len), B.half_len);
        double b = fmin(fmax(-dot(r, d), 0.0), B.b_back);
        double xc[3], df[3];
        for (int i = 0; i < 3; i++) {
            xc[i] = xe[i] + a * e[i] - b * d[i];
            df[i] = x[i] - xc[i];
        }
        const double dist = sqrt(dot(df, df));
        double nb[3];
        for (int i = 0; i < 3; i++) nb[i] = dist > 0.0 ? df[i] / dist : n[i];
        double arm[3] = {xc[0] - xB[0], xc[1] - xB[1], xc[2] - xB[2]};
        double w[3] = {T.wB[0], T.wB[1], T.wB[2]}, wxr[3];
        cross(w, arm, wxr);
        double vrel[3];
        for (int i = 0; i < 3; i++) vrel[i] = v[i] - (T.vB[i] + wxr[i]);
        const double phihat = dist - R + dt * fmin(dot(vrel, nb), 0.0);
        const bool touch = phihat < 0.0;
        // the brick: this particle at one extreme, a few others inside its box
        float fx[3] = {(float)x[0], (float)x[1], (float)x[2]};
        float bb[7] = {fx[0], fx[1], fx[2], fx[0], fx[1], fx[2], (float)vmax_p};
        for (int q = 0; q < 4; q++)
            for (int k = 0; k < 3; k++) {
                float o = fx[k] + (float)(urand() * 0.006) * (((trial >> (k + 1)) & 1) ? 1.0f : -1.0f);
                bb[k] = fminf(bb[k], o);
                bb[3 + k] = fmaxf(bb[3 + k], o);
            }
        bb[6] = nextafterf(bb[6], INFINITY);
        const bool keep = brick_near_tool(bb, T, Rmax, dt, jdt);
        if (touch) {
            contact++;
            if (!keep) {
                missed++;
                if (missed <= 5)
                    printf("miss trial %d where %d dist %.6g phihat %.6g\n", trial, where, dist, phihat);
            }
            DevTool T0 = T;
            T0.wB[0] = T0.wB[1] = T0.wB[2] = 0.0f;
            if (!brick_near_tool(bb, T0, Rmax, dt, jdt)) norot_missed++;
        } else {
            double vb = sqrt(dot(T.vB, T.vB));
            double arm0[3] = {xe[0] - xB[0], xe[1] - xB[1], xe[2] - xB[2]};
            double reach = Rmax + dt * (bb[6] + vb + wn * (sqrt(dot(arm0, arm0)) + B.half_len + B.b_back)) + 1e-5;
            if (!keep && bbox_only(bb, T, reach, jdt)) pruned++;
        }
    }
    printf("cases %ld contact %ld missed %ld norot_missed %ld pruned %ld\n", cases, contact, missed, norot_missed,
           pruned);
    return missed ? 1 : 0;
}
