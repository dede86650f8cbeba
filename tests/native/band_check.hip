// Host-side check of the label pass's brick skip test (tlmpm_band.h): for
// particles placed on the faces of the blade band (Eq. 4) with FP32 state whose
// rounded position fl(X + u) lies up to half an ulp away from the exact X + u that
// label_digit reads, a brick whose particle gets a digit must never be skipped.
// Prints "cases <n> labelled <k> outside <o> unwidened_missed <u> missed <m>":
// o counts labelled cases whose exact position lies more than 1e-9 m outside the
// FP32 box, u the labelled cases that the same test on the box without the ulp
// widening would skip (the box shrunk by one ulp per face is passed, which the
// widening turns back into the plain FP32 box); m must be 0.  Runs on the CPU
// only (no HIP runtime call).
#include <math.h>
#include <stdint.h>
#include <stdio.h>

#include "../../paper_2609_27342_amd/csrc/tlmpm_band.h"

static uint64_t g_state = 0x9E3779B97F4A7C15ull;
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

int main()
{
    long cases = 0, labelled = 0, outside = 0, missed = 0, unwidened_missed = 0;
    const double dt = 1e-4;
    for (int trial = 0; trial < 200000; trial++) {
        // FP32 state: X in [0.05, 0.3] per axis (large coordinates give large ulps),
        // u either tiny (so fl(X + u) rounds to a neighbour of X) or O(1 mm)
        float X[3], u[3], v[3];
        for (int a = 0; a < 3; a++) {
            X[a] = (float)(0.05 + 0.25 * urand());
            double scale = (trial & 1) ? 1e-8 : 1e-3;
            u[a] = (float)((urand() - 0.5) * 2.0 * scale);
            v[a] = (float)((urand() - 0.5) * 0.4);
        }
        double x[3], xv[3];
        float fx[3];
        for (int a = 0; a < 3; a++) {
            x[a] = (double)X[a] + (double)u[a]; // what label_digit reads
            fx[a] = X[a] + u[a];                // what the brick box holds
            xv[a] = (double)v[a];
        }
        // a blade frame in a random orientation (or axis-aligned, where the FP32
        // error along the normal is largest)
        double n[3], d[3], e[3];
        if (trial % 4 == 0) {
            int ax = (trial / 4) % 3;
            n[0] = n[1] = n[2] = 0.0;
            n[ax] = (trial & 8) ? 1.0 : -1.0;
            d[0] = d[1] = d[2] = 0.0;
            d[(ax + 1) % 3] = -1.0;
        } else {
            double r[3] = {urand() - 0.5, urand() - 0.5, urand() - 0.5}, t[3] = {urand() - 0.5, urand() - 0.5, urand() - 0.5};
            unit(r);
            double k = t[0] * r[0] + t[1] * r[1] + t[2] * r[2];
            for (int i = 0; i < 3; i++) t[i] -= k * r[i];
            unit(t);
            for (int i = 0; i < 3; i++) {
                n[i] = r[i];
                d[i] = t[i];
            }
        }
        cross(n, d, e);
        DevBlade B;
        B.half_width = 0.012 + 0.01 * urand();
        B.half_len = 0.05 + 0.05 * urand();
        B.b_back = 0.02 + 0.03 * urand();
        B.b_lead = 0.002;
        for (int i = 0; i < 3; i++) {
            B.n[i] = n[i];
            B.d[i] = d[i];
            B.e[i] = e[i];
            B.ve[i] = -0.2 * d[i];
        }
        B.cut = 0;
        B.new_cut = 0;
        // place the particle on one band face: s = +-h, l = +-L, f = 0 or the rear
        // face, the other two coordinates strictly inside
        const int face = trial % 6;
        double s = (urand() - 0.5) * B.half_width, l = (urand() - 0.5) * B.half_len, f = -urand() * 0.5 * B.b_back;
        double uc = (B.ve[0] - xv[0]) * d[0] + (B.ve[1] - xv[1]) * d[1] + (B.ve[2] - xv[2]) * d[2];
        switch (face) {
        case 0: s = B.half_width; break;
        case 1: s = -B.half_width; break;
        case 2: l = B.half_len; break;
        case 3: l = -B.half_len; break;
        case 4: f = 0.0; break;
        default: f = -B.b_back - fmax(uc * dt, 0.0); break;
        }
        // tiny offsets around the face, a few ulps of the position
        double jit = (urand() - 0.5) * 6e-8;
        if (face < 2) s += jit;
        else if (face < 4) l += jit;
        else f += jit;
        for (int i = 0; i < 3; i++) B.xe[i] = x[i] - (s * n[i] + l * e[i] + f * d[i]);
        cases++;
        int dg = label_digit(x, xv, B, dt);
        if (!dg) continue;
        labelled++;
        // a brick: this particle at one extreme, a few others inside its box
        float bb[7] = {fx[0], fx[1], fx[2], fx[0], fx[1], fx[2], 0.0f};
        for (int q = 0; q < 4; q++)
            for (int a = 0; a < 3; a++) {
                float o = fx[a] + (float)(urand() * 0.004) * ((trial >> (a + 1)) & 1 ? 1.0f : -1.0f);
                bb[a] = fminf(bb[a], o);
                bb[3 + a] = fmaxf(bb[3 + a], o);
            }
        bb[6] = sqrtf(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        // does the exact position lie outside the unwidened FP32 box?
        double out = 0.0;
        for (int a = 0; a < 3; a++) out = fmax(out, fmax((double)bb[a] - x[a], x[a] - (double)bb[3 + a]));
        if (out > 1e-9) outside++;
        float shrunk[7];
        for (int a = 0; a < 3; a++) {
            shrunk[a] = nextafterf(bb[a], INFINITY);
            shrunk[3 + a] = nextafterf(bb[3 + a], -INFINITY);
        }
        shrunk[6] = bb[6];
        if (!brick_near_band(shrunk, B, dt)) unwidened_missed++;
        if (!brick_near_band(bb, B, dt)) {
            missed++;
            if (missed <= 5)
                printf("miss trial %d face %d x %.17g %.17g %.17g out %.3g\n", trial, face, x[0], x[1], x[2], out);
        }
    }
    printf("cases %ld labelled %ld outside %ld unwidened_missed %ld missed %ld\n", cases, labelled, outside,
           unwidened_missed, missed);
    return missed ? 1 : 0;
}
