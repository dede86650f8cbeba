// Host-side check of the material-contact search skip (tlmpm_reach.h,
// pair_skip_bounds_ok): a candidate the rule lets skip must have no partner, i.e.
// every particle within the bin edge hb (FP32 reach test, as in the pair search) is
// a reference neighbour (reference cells at most one apart per axis, FP64 floor of
// (X - origin) / dx) with a compatible side code.
//
// Each trial builds a body of 6 x 6 x 4 bricks (4 x 4 x 4 cells, 8 jittered
// particles per cell) and a second piece of 2 x 2 x 2 bricks one empty brick beyond
// the body's +x face in the reference configuration, which two trials in three push
// against that face, to a gap below hb (foreign contact: no reference neighbours).
// Displacements: a translation, a small rotation, a strain and noise, with
// amplitudes drawn across the rule's thresholds, and in one trial in five a slip: the
// body's upper half slides along x by 0.5 to 1.5 dx over the lower one (unlabelled,
// so that only the neighbour bound can keep pairs across the slip plane searched).
// Side codes from a random cut plane (digit 1 or 2 within a band about it, 0
// elsewhere; none in slip trials).  The per-brick anchors
// and spreads are formed as the transfer pass forms them: the anchor is the centre
// of the brick's box of the previous positions fl(X + u0) minus the centre of its
// box of reference positions, the spread the largest |u - a| (FP32).
// Usage: pair_skip_check [mode]; mode 0 is the rule as built, mode 1 loosens the
// foreign-brick bound (4 dx -> 8 dx), mode 2 the neighbour bound (dx -> 2 dx).
// Prints "trials <t> candidates <n> skipped <s> violations <v>"; mode 0 must give
// v = 0 with s > 0, the loosened modes must give v > 0.  CPU only.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <unordered_map>
#include <vector>

#include "../../paper_2609_27342_amd/csrc/tlmpm_reach.h"

static uint64_t g_state = 0x9E3779B97F4A7C15ull;
static double urand()
{
    g_state ^= g_state << 13;
    g_state ^= g_state >> 7;
    g_state ^= g_state << 17;
    return (double)(g_state >> 11) * (1.0 / 9007199254740992.0);
}

static bool conflict(uint32_t a, uint32_t b)
{
    uint32_t a1 = a & 0x7FFFu, a2 = (a >> 15) & 0x7FFFu, b1 = b & 0x7FFFu, b2 = (b >> 15) & 0x7FFFu;
    return ((a1 & b2) | (a2 & b1)) != 0u;
}

struct Brick {
    float lo[3], hi[3], rlo[3], rhi[3], a[3], s;
    uint32_t orr;
};

static bool loosened_ok(int mode, const float U[3], const float Dk[3], float hb, float dx, float M)
{
    if (mode == 0) return pair_skip_bounds_ok(U, Dk, hb, dx, M);
    if (mode == 1) { // the foreign-brick bound at 8 dx instead of 4 dx
        const float half[3] = {U[0] * 0.5f - hb * 0.5f, U[1] * 0.5f - hb * 0.5f, U[2] * 0.5f - hb * 0.5f};
        const float Uz[3] = {0.0f, 0.0f, 0.0f};
        for (int k = 0; k < 3; k++)
            if (!(half[k] + hb <= 4.0f * dx)) return false; // U + hb <= 8 dx
        return pair_skip_bounds_ok(Uz, Dk, hb, dx, M);
    }
    const float Dh[3] = {Dk[0] * 0.5f - hb * 0.5f, Dk[1] * 0.5f - hb * 0.5f, Dk[2] * 0.5f - hb * 0.5f};
    return pair_skip_bounds_ok(U, Dh, hb, dx, M); // Dk + hb <= 2 dx
}

int main(int argc, char** argv)
{
    const int mode = argc > 1 ? atoi(argv[1]) : 0;
    const double dx = 1e-3, org[3] = {0.1, 0.2, 0.05};
    long trials = 0, cands = 0, skipped = 0, violations = 0;
    for (int trial = 0; trial < 60; trial++) {
        trials++;
        // reference particles: body bricks (0..5, 0..5, 0..3), piece bricks (7..8, 1..2, 1..2)
        std::vector<float> X;
        std::vector<int> cellv, brk;
        std::unordered_map<long long, int> bid;
        auto bkey = [](int i, int j, int k) { return ((long long)i * 4096 + j) * 4096 + k; };
        std::vector<Brick> B;
        auto add_brick = [&](int bi, int bj, int bk) {
            const int id = (int)B.size();
            bid[bkey(bi, bj, bk)] = id;
            B.push_back(Brick{});
            for (int c = 0; c < 64; c++) {
                const int cx = bi * 4 + (c & 3), cy = bj * 4 + ((c >> 2) & 3), cz = bk * 4 + (c >> 4);
                for (int q = 0; q < 8; q++) {
                    double p[3] = {cx + 0.25 + 0.5 * (q & 1), cy + 0.25 + 0.5 * ((q >> 1) & 1), cz + 0.25 + 0.5 * (q >> 2)};
                    for (int a = 0; a < 3; a++) {
                        p[a] += (urand() - 0.5) * 0.4;
                        X.push_back((float)(org[a] + p[a] * dx));
                    }
                    cellv.push_back(0);
                    brk.push_back(id);
                }
            }
        };
        for (int i = 0; i < 6; i++)
            for (int j = 0; j < 6; j++)
                for (int k = 0; k < 4; k++) add_brick(i, j, k);
        for (int i = 7; i < 9; i++)
            for (int j = 1; j < 3; j++)
                for (int k = 1; k < 3; k++) add_brick(i, j, k);
        const size_t n = brk.size();
        std::vector<int> cell(3 * n);
        for (size_t p = 0; p < n; p++)
            for (int a = 0; a < 3; a++) cell[3 * p + a] = (int)floor(((double)X[3 * p + a] - org[a]) / dx);
        // displacements: the kind of trial sets the amplitudes (across the thresholds)
        const int kind = trial % 4;
        const double amp = dx * (kind == 0 ? 0.01 : kind == 1 ? 0.1 : kind == 2 ? 0.3 : 1.0) * (0.5 + urand());
        double t[3], w[3], e[3];
        for (int a = 0; a < 3; a++) {
            t[a] = (urand() - 0.5) * 20.0 * dx; // translation (no effect on the rule)
            w[a] = (urand() - 0.5) * amp / (20.0 * dx); // rotation angle ~ amp over the body
            e[a] = (urand() - 0.5) * amp / (20.0 * dx);
        }
        const bool press = (trial % 3) != 0; // the piece pushed against the body's +x face
        const double cb[3] = {org[0] + 12 * dx, org[1] + 12 * dx, org[2] + 8 * dx};
        const float hb = (float)(dx * (0.3 + 0.6 * urand()));
        const double gap = hb * urand(); // between the piece's and the body's faces
        const bool slip = trial % 5 == 4;
        const double slip_d = dx * (0.5 + urand());
        std::vector<float> u(3 * n), u0(3 * n), x(3 * n), x0(3 * n);
        for (size_t p = 0; p < n; p++) {
            double r[3], up[3];
            for (int a = 0; a < 3; a++) r[a] = (double)X[3 * p + a] - cb[a];
            up[0] = t[0] + w[1] * r[2] - w[2] * r[1] + e[0] * r[0];
            up[1] = t[1] + w[2] * r[0] - w[0] * r[2] + e[1] * r[1];
            up[2] = t[2] + w[0] * r[1] - w[1] * r[0] + e[2] * r[2];
            for (int a = 0; a < 3; a++) up[a] += (urand() - 0.5) * amp * 0.2;
            if (slip && r[2] > 0.0) up[0] += slip_d;
            if (brk[p] >= 144 && press) {
                // piece: its face at reference x = 28 dx moved to the body's face at 24 dx
                // plus the gap (a translation of the piece alone)
                up[0] = -4.0 * dx + gap + (urand() - 0.5) * 1e-3 * dx;
                up[1] = (urand() - 0.5) * 1e-3 * dx;
                up[2] = (urand() - 0.5) * 1e-3 * dx;
            }
            for (int a = 0; a < 3; a++) {
                u[3 * p + a] = (float)up[a];
                u0[3 * p + a] = (float)(up[a] - (urand() - 0.5) * 1e-3 * dx);
                x[3 * p + a] = X[3 * p + a] + u[3 * p + a];
                x0[3 * p + a] = X[3 * p + a] + u0[3 * p + a];
            }
        }
        // side codes: a cut plane through the body, digits within a band about it
        double nrm[3] = {urand() - 0.5, urand() - 0.5, urand() - 0.5}, nn = 0.0;
        for (int a = 0; a < 3; a++) nn += nrm[a] * nrm[a];
        for (int a = 0; a < 3; a++) nrm[a] /= sqrt(nn);
        std::vector<uint32_t> key(n, 0u);
        const double band = dx * (1.0 + 6.0 * urand());
        for (size_t p = 0; p < n; p++) {
            double s = 0.0;
            for (int a = 0; a < 3; a++) s += ((double)X[3 * p + a] - cb[a]) * nrm[a];
            if (fabs(s) < band && !slip) key[p] = s < 0.0 ? 1u : (1u << 15);
        }
        // per brick: boxes, anchors and spreads as the transfer pass forms them
        for (auto& b : B)
            for (int a = 0; a < 3; a++) {
                b.lo[a] = b.rlo[a] = 1e30f;
                b.hi[a] = b.rhi[a] = -1e30f;
                b.orr = 0u;
            }
        for (size_t p = 0; p < n; p++) {
            Brick& b = B[brk[p]];
            for (int a = 0; a < 3; a++) {
                b.lo[a] = fminf(b.lo[a], x0[3 * p + a]);
                b.hi[a] = fmaxf(b.hi[a], x0[3 * p + a]);
                b.rlo[a] = fminf(b.rlo[a], X[3 * p + a]);
                b.rhi[a] = fmaxf(b.rhi[a], X[3 * p + a]);
            }
            b.orr |= key[p];
        }
        for (auto& b : B) {
            for (int a = 0; a < 3; a++) b.a[a] = 0.5f * (b.lo[a] + b.hi[a]) - 0.5f * (b.rlo[a] + b.rhi[a]);
            b.s = 0.0f;
        }
        for (size_t p = 0; p < n; p++) {
            Brick& b = B[brk[p]];
            for (int a = 0; a < 3; a++) b.s = fmaxf(b.s, fabsf(u[3 * p + a] - b.a[a]));
        }
        float U[3];
        for (int a = 0; a < 3; a++) {
            float mx = -1e30f, mn = 1e30f;
            for (auto& b : B) {
                mx = fmaxf(mx, b.a[a] + b.s);
                mn = fminf(mn, b.a[a] - b.s);
            }
            U[a] = mx - mn;
        }
        // brick coordinates back from the map
        std::vector<int> bc(3 * B.size());
        for (auto& kv : bid) {
            long long k = kv.first;
            bc[3 * kv.second + 2] = (int)(k % 4096);
            bc[3 * kv.second + 1] = (int)((k / 4096) % 4096);
            bc[3 * kv.second + 0] = (int)(k / (4096LL * 4096));
        }
        std::vector<char> bskip(B.size());
        std::vector<uint32_t> born(B.size());
        for (size_t i = 0; i < B.size(); i++) {
            float Dk[3] = {0.0f, 0.0f, 0.0f}, M = 0.0f;
            uint32_t o = 0u;
            for (int d = 0; d < 27; d++) {
                auto it = bid.find(bkey(bc[3 * i] + d % 3 - 1, bc[3 * i + 1] + (d / 3) % 3 - 1, bc[3 * i + 2] + d / 9 - 1));
                if (it == bid.end()) continue;
                const Brick& q = B[it->second];
                for (int a = 0; a < 3; a++) Dk[a] = fmaxf(Dk[a], fabsf(q.a[a] - B[i].a[a]) + q.s);
                o |= q.orr;
            }
            for (int a = 0; a < 3; a++) {
                Dk[a] += B[i].s;
                M = fmaxf(M, fmaxf(fabsf(B[i].lo[a]), fabsf(B[i].hi[a])));
            }
            bskip[i] = loosened_ok(mode, U, Dk, hb, (float)dx, M);
            born[i] = o;
        }
        // brute force over pairs within hb (hash grid of edge hb on the current positions)
        std::unordered_map<long long, std::vector<int>> grid;
        auto gk = [&](int i, int j, int k) { return ((long long)(i + 100000) * 200000 + (j + 100000)) * 200000 + (k + 100000); };
        std::vector<int> gc(3 * n);
        for (size_t p = 0; p < n; p++) {
            for (int a = 0; a < 3; a++) gc[3 * p + a] = (int)floorf(x[3 * p + a] / hb);
            grid[gk(gc[3 * p], gc[3 * p + 1], gc[3 * p + 2])].push_back((int)p);
        }
        for (size_t p = 0; p < n; p++) {
            cands++;
            const int b = brk[p];
            if (!(bskip[b] && !conflict(key[p], born[b]))) continue;
            skipped++;
            bool bad = false;
            for (int d = 0; d < 27 && !bad; d++) {
                auto it = grid.find(gk(gc[3 * p] + d % 3 - 1, gc[3 * p + 1] + (d / 3) % 3 - 1, gc[3 * p + 2] + d / 9 - 1));
                if (it == grid.end()) continue;
                for (int q : it->second) {
                    if ((size_t)q == p) continue;
                    const float ex = x[3 * p] - x[3 * q], ey = x[3 * p + 1] - x[3 * q + 1], ez = x[3 * p + 2] - x[3 * q + 2];
                    if (ex * ex + ey * ey + ez * ez >= hb * hb) continue;
                    const bool near = abs(cell[3 * p] - cell[3 * q]) <= 1 && abs(cell[3 * p + 1] - cell[3 * q + 1]) <= 1 &&
                                      abs(cell[3 * p + 2] - cell[3 * q + 2]) <= 1;
                    if (!near || conflict(key[p], key[q])) {
                        bad = true;
                        break;
                    }
                }
            }
            if (bad) {
                violations++;
                if (mode == 0 && violations <= 5) printf("violation trial %d particle %zu\n", trial, p);
            }
        }
    }
    printf("trials %ld candidates %ld skipped %ld violations %ld\n", trials, cands, skipped, violations);
    return (mode == 0 && violations) ? 1 : 0;
}
