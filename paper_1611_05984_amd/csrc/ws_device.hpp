// ws_device.hpp -- device-side data and helpers of the gfx950 time step.
//
// State is kept as eta = w - w_s (free surface), P, Q in FP32 structure-of-
// arrays fields of nyp rows x pitch floats (x fastest, rows padded to whole
// tiles).  Bathymetry is kept as the still-water depth at the corners,
// D = w_s - z (unclamped), so that every kernel works with depths measured
// from the still water level and a lake at rest is all zeros.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ws {

constexpr int TX = 64;        // tile width  (cells along x) = row segment length
constexpr int TY = 16;        // tile height (cells along y) = column segment length
constexpr int NT = 256;       // threads per tile workgroup (4 wave64)
constexpr int MAXC = 256;     // wave components per side
constexpr int TABW = 8;       // doubles per component: a, omega, kx, ky, cx, cy, phase, -
constexpr int NRED_MAX = 2048;  // reduced unknowns per row/column system

enum { BC_SOLID = 0, BC_SPONGE = 1, BC_WAVES = 2 };
enum { BSNQ = 0, NLSW = 1 };
enum { FRIC_NONE = 0, FRIC_QUAD = 1, FRIC_MANNING = 2 };

struct SideDev {
    int type, width, ncomp, pad;
    const double *tab;  // ncomp * TABW
};

struct Dom {
    int nx, ny, pitch, zpitch;
    int nu, nv;         // reduced unknowns of one row / one column system
    int model, friction;
    float dx, dy, rdx, rdy;
    float g, Bd, theta, eps, fcoef;
    const float *D;     // corner still-water depth, (ny+1) rows x zpitch
    SideDev side[4];
};

__device__ __forceinline__ bool is_wall(const Dom &d, int s) { return d.side[s].type != BC_WAVES; }

// Corner index behind a side: mirrored across walls and sponges, held at the
// boundary value across wave makers; clamped into range for padding cells.
__device__ __forceinline__ int map_corner(int c, int n, bool lo_wall, bool hi_wall) {
    if (c < 0) c = lo_wall ? -c : 0;
    if (c > n) c = hi_wall ? 2 * n - c : n;
    return c < 0 ? 0 : (c > n ? n : c);
}

__device__ __forceinline__ float corner_D(const Dom &d, int ci, int cj) {
    int i = map_corner(ci, d.nx, is_wall(d, 0), is_wall(d, 1));
    int j = map_corner(cj, d.ny, is_wall(d, 2), is_wall(d, 3));
    return d.D[(size_t)j * d.zpitch + i];
}

// Wave-maker values at (x, y, t): sum of a sin(omega t + phi - kx x - ky y),
// discharges c cos(theta) eta, c sin(theta) eta per component.  The phase is
// formed and reduced to [-pi, pi] in double, the sine taken in single.
__device__ inline void wave_eval(const SideDev &s, double x, double y, double t, float &e,
                                 float &p, float &q) {
    float se = 0.f, sp = 0.f, sq = 0.f;
    for (int m = 0; m < s.ncomp; ++m) {
        const double *c = s.tab + TABW * m;
        double ph = c[1] * t + c[6] - (c[2] * x + c[3] * y);
        ph -= 6.283185307179586 * rint(ph * 0.15915494309189535);
        float v = (float)c[0] * sinf((float)ph);
        se += v;
        sp += (float)c[4] * v;
        sq += (float)c[5] * v;
    }
    e = se;
    p = sp;
    q = sq;
}

// Value of cell (i, j), inside or in the two-cell ghost ring: reflected across
// every wall side first (normal discharge of that side changes sign), then, if
// still behind a wave-maker side, that maker's values at the reflected
// position.  Cells further out (tile padding) are clamped into the domain.
__device__ inline void load_cell(const Dom &d, const float *__restrict__ E,
                                 const float *__restrict__ P, const float *__restrict__ Q, int i,
                                 int j, double t, float &e, float &p, float &q) {
    float sp = 1.f, sq = 1.f;
    if (i < 0 && is_wall(d, 0)) { i = -1 - i; sp = -sp; }
    if (i >= d.nx && is_wall(d, 1)) { i = 2 * d.nx - 1 - i; sp = -sp; }
    if (j < 0 && is_wall(d, 2)) { j = -1 - j; sq = -sq; }
    if (j >= d.ny && is_wall(d, 3)) { j = 2 * d.ny - 1 - j; sq = -sq; }
    const bool in_i = i >= 0 && i < d.nx, in_j = j >= 0 && j < d.ny;
    int side = -1;
    if (!in_i) side = i < 0 ? 0 : 1;
    else if (!in_j) side = j < 0 ? 2 : 3;
    if (side >= 0 && d.side[side].type == BC_WAVES) {
        wave_eval(d.side[side], (i + 0.5) * (double)d.dx, (j + 0.5) * (double)d.dy, t, e, p, q);
    } else {
        i = i < 0 ? 0 : (i >= d.nx ? d.nx - 1 : i);
        j = j < 0 ? 0 : (j >= d.ny ? d.ny - 1 : j);
        size_t k = (size_t)j * d.pitch + i;
        e = E[k];
        p = P[k];
        q = Q[k];
    }
    p *= sp;
    q *= sq;
}

// ---------------------------------------------------------------- KP07 parts
__device__ __forceinline__ float minmod3(float a, float b, float c) {
    if (a > 0.f && b > 0.f && c > 0.f) return fminf(a, fminf(b, c));
    if (a < 0.f && b < 0.f && c < 0.f) return fmaxf(a, fmaxf(b, c));
    return 0.f;
}

struct F3 { float e, n, t; };  // surface, normal and tangential discharge at a face

// Limited linear reconstruction of one cell along one direction, then the
// conservative positivity correction of the surface against the depths of
// the cell's low/high faces (w < B  <=>  eta < -D).
__device__ __forceinline__ void reconstruct(float em, float e0, float ep, float nm, float n0,
                                            float np, float tm, float t0, float tp, float Dlo,
                                            float Dhi, float th, F3 &lo, F3 &hi) {
    float se = minmod3(th * (e0 - em), 0.5f * (ep - em), th * (ep - e0));
    float sn = minmod3(th * (n0 - nm), 0.5f * (np - nm), th * (np - n0));
    float st = minmod3(th * (t0 - tm), 0.5f * (tp - tm), th * (tp - t0));
    lo.e = e0 - 0.5f * se;
    hi.e = e0 + 0.5f * se;
    lo.n = n0 - 0.5f * sn;
    hi.n = n0 + 0.5f * sn;
    lo.t = t0 - 0.5f * st;
    hi.t = t0 + 0.5f * st;
    if (hi.e < -Dhi) {
        hi.e = -Dhi;
        lo.e = 2.f * e0 + Dhi;
    } else if (lo.e < -Dlo) {
        lo.e = -Dlo;
        hi.e = 2.f * e0 + Dlo;
    }
}

// Desingularized velocity sqrt(2) h m / sqrt(h^4 + max(h^4, eps)).
__device__ __forceinline__ float desing(float h, float m, float eps) {
    float h2 = h * h, h4 = h2 * h2;
    return 1.41421356237f * h * m * rsqrtf(h4 + fmaxf(h4, eps));
}

// Central-upwind flux at a face in well-balanced ("pre-balanced") form.  With
// D_f the face still-water depth and h = eta + D_f, the pressure g h^2/2 is
// split into g eta (eta + 2 D_f)/2 + g D_f^2/2; the constant g D_f^2/2 passes
// through the central-upwind average unchanged and cancels exactly against
// the matching part of the bottom source, so it is dropped here and the
// source becomes g (D_hi - D_lo)/dx * eta_cell.  Where both sides are dry the
// face flux of the original form is zero, i.e. (0, -g D_f^2/2, 0) here.
// Returns (mass, normal momentum, tangential momentum).
__device__ __forceinline__ void cu_flux(float g, float eps, float Df, const F3 &L, const F3 &R,
                                        float &H0, float &H1, float &H2) {
    float hL = fmaxf(L.e + Df, 0.f), hR = fmaxf(R.e + Df, 0.f);
    float uL = desing(hL, L.n, eps), vL = desing(hL, L.t, eps);
    float uR = desing(hR, R.n, eps), vR = desing(hR, R.t, eps);
    float nL = hL * uL, tL = hL * vL, nR = hR * uR, tR = hR * vR;
    float cL = sqrtf(g * hL), cR = sqrtf(g * hR);
    float ap = fmaxf(fmaxf(uL + cL, uR + cR), 0.f);
    float am = fminf(fminf(uL - cL, uR - cR), 0.f);
    if (ap - am <= 1e-10f) {
        H0 = 0.f;
        H1 = -0.5f * g * Df * Df;
        H2 = 0.f;
        return;
    }
    float eL = hL > 0.f ? L.e : -Df, eR = hR > 0.f ? R.e : -Df;
    float pL = 0.5f * g * eL * (eL + 2.f * Df), pR = 0.5f * g * eR * (eR + 2.f * Df);
    float inv = 1.f / (ap - am), apam = ap * am * inv;
    H0 = (ap * nL - am * nR) * inv + apam * (R.e - L.e);
    H1 = (ap * (nL * uL + pL) - am * (nR * uR + pR)) * inv + apam * (nR - nL);
    H2 = (ap * (nL * vL) - am * (nR * vR)) * inv + apam * (tR - tL);
}

// Row/column system coefficients of eq. 23 for one cell.
__device__ __forceinline__ void tri_coef(const Dom &d, float dep, float ddep, float rh, float &A,
                                         float &B, float &C) {
    if (d.model == NLSW) {
        A = 0.f;
        B = 1.f;
        C = 0.f;
        return;
    }
    float al = (d.Bd + 1.f / 3.f) * dep * dep * rh * rh;
    float be = dep * ddep * rh * (1.f / 6.f);
    A = be - al;
    B = 1.f + 2.f * al;
    C = -be - al;
}

__device__ __forceinline__ float sponge_gamma(float dist, float Ls) {
    return dist >= Ls ? 1.f : 0.5f * (1.f + cosf(3.14159265358979f * (Ls - dist) / Ls));
}

}  // namespace ws
