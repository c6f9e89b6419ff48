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

constexpr int TX = 64;        // solver tile width  (cells along x)
constexpr int TY = 16;        // solver tile height (cells along y) = column segment length
constexpr int MX = 16;        // row segment length (4 per solver tile row)
constexpr int NT = 256;       // threads per solver tile workgroup (4 wave64)
constexpr int NTB = 128;      // the same in the batch (2 wave64)
constexpr int SO = 62;        // stencil: output columns per 64-lane strip wave
constexpr int SY = 32;        // stencil: rows streamed per strip wave
constexpr int SWG = 4;        // stencil: strip waves per workgroup
constexpr int MAXC = 256;     // wave components per side
constexpr int TABW = 8;       // doubles per component: a, omega, kx, ky, cx, cy, phase, -
constexpr int NRED_MAX = 2048;  // reduced unknowns per row/column system

enum { BC_SOLID = 0, BC_SPONGE = 1, BC_WAVES = 2 };
enum { BSNQ = 0, NLSW = 1 };
enum { FRIC_NONE = 0, FRIC_QUAD = 1, FRIC_MANNING = 2 };

struct SideDev {
    int type, width, ncomp;
    float expo;         // sponge: exponent s of the damping factor gamma^s (1 = eq. 30)
    const double *tab;  // ncomp * TABW
};

struct Dom {
    int nx, ny, pitch, zpitch;
    int nu, nv;         // reduced unknowns of one row / one column system
    int model, friction;
    int gl;             // ghost-buffer positions per layer: max(nx, ny) + 4
    float dx, dy, rdx, rdy;
    float g, Bd, theta, eps, fcoef;
    const float *D;     // corner still-water depth, (ny+1) rows x zpitch
    const float *gh;    // wave-maker ghost values at the pass's time (see ghost_index)
    SideDev side[4];
};

// Wave-maker ghost values are precomputed per time level: [side][layer][pos][eta, P, Q],
// layer 0 next to the boundary, pos = along-side cell index + 2 (covers -2 .. n+1).
__device__ __forceinline__ size_t ghost_index(const Dom &d, int side, int layer, int pos) {
    return (((size_t)side * 2 + layer) * d.gl + pos) * 3;
}

__device__ __forceinline__ bool is_wall(const Dom &d, int s) { return d.side[s].type != BC_WAVES; }

// Side type by a run-time side index, as selects: keeps a Dom held in
// registers free of dynamic indexing.
__device__ __forceinline__ int side_type(const Dom &d, int s) {
    return s == 0 ? d.side[0].type : s == 1 ? d.side[1].type : s == 2 ? d.side[2].type : d.side[3].type;
}

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
// Components first, first + stride, ... of the sum (one lane's share).
__device__ inline void wave_partial(const SideDev &s, double x, double y, double t, int first, int stride,
                                    float &se, float &sp, float &sq) {
    for (int m = first; m < s.ncomp; m += stride) {
        const double *c = s.tab + TABW * m;
        double ph = c[1] * t + c[6] - (c[2] * x + c[3] * y);
        ph -= 6.283185307179586 * rint(ph * 0.15915494309189535);
        const float v = (float)c[0] * sinf((float)ph);
        se += v;
        sp += (float)c[4] * v;
        sq += (float)c[5] * v;
    }
}

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
// position (precomputed ghost buffer).  Cells further out (padding) are
// clamped into the domain.
__device__ inline void load_cell(const Dom &d, const float *__restrict__ E,
                                 const float *__restrict__ P, const float *__restrict__ Q, int i,
                                 int j, float &e, float &p, float &q) {
    float sp = 1.f, sq = 1.f;
    if (i < 0 && is_wall(d, 0)) { i = -1 - i; sp = -sp; }
    if (i >= d.nx && is_wall(d, 1)) { i = 2 * d.nx - 1 - i; sp = -sp; }
    if (j < 0 && is_wall(d, 2)) { j = -1 - j; sq = -sq; }
    if (j >= d.ny && is_wall(d, 3)) { j = 2 * d.ny - 1 - j; sq = -sq; }
    const bool in_i = i >= 0 && i < d.nx, in_j = j >= 0 && j < d.ny;
    int side = -1;
    if (!in_i) side = i < 0 ? 0 : 1;
    else if (!in_j) side = j < 0 ? 2 : 3;
    if (side >= 0 && side_type(d, side) == BC_WAVES) {
        int layer = side == 0 ? -1 - i : side == 1 ? i - d.nx : side == 2 ? -1 - j : j - d.ny;
        int pos = (side < 2 ? j : i) + 2;
        layer = layer < 0 ? 0 : (layer > 1 ? 1 : layer);
        pos = pos < 0 ? 0 : (pos >= d.gl ? d.gl - 1 : pos);
        const float *g = d.gh + ghost_index(d, side, layer, pos);
        e = g[0];
        p = g[1];
        q = g[2];
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
// minmod of three: the smallest if all are positive, the largest if all are
// negative, else 0 -- the median of (min, max, 0) (v_med3: three
// instructions with v_min3 and v_max3).
__device__ __forceinline__ float minmod3(float a, float b, float c) {
    const float mn = fminf(a, fminf(b, c)), mx = fmaxf(a, fmaxf(b, c));
    return __builtin_amdgcn_fmed3f(mn, mx, 0.f);
}

// Hardware reciprocal, reciprocal square root and square root (1 ulp); their
// arguments here are never denormal except sqrt of a vanishing depth.
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Lane shifts across the 64-lane wave (DPP wave_shr:1 / wave_shl:1): lane k
// takes lane k-1 (shr) or k+1 (shl); the lane without a source takes `old`.
__device__ __forceinline__ float shr1(float v, float old) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float shl1(float v, float old) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), 0x130, 0xf, 0xf, false));
}
// The same shifts where the edge lane's result is never used (it belongs to
// a halo lane): the vacated lane reads 0 (bound_ctrl), so the shift is one
// DPP move with no copy of an "old" value first.
__device__ __forceinline__ float shr1z(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float shl1z(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}

struct F3 { float e, n, t; };  // surface, normal and tangential discharge at a face

// Reconstruction constants of the generalized minmod limiter with parameter
// theta: minmod(theta a, c/2, theta b) = theta minmod(a, c/(2 theta), b) for
// theta > 0, and the face values take half the slope, so the limiter runs on
// the plain differences with the central one scaled by kc = 1/(2 theta), and
// the face values add or subtract hth = theta/2 times its result (two
// multiplies fewer a variable).
struct Recon { float kc, hth; };
__device__ __forceinline__ Recon recon_k(float th) { return {0.5f / th, 0.5f * th}; }

// Limited linear reconstruction of one cell along one direction, then the
// conservative positivity correction of the surface against the depths of
// the cell's low/high faces (w < B  <=>  eta < -D).
__device__ __forceinline__ void reconstruct(float em, float e0, float ep, float nm, float n0,
                                            float np, float tm, float t0, float tp, float Dlo,
                                            float Dhi, Recon rk, F3 &lo, F3 &hi) {
    const float me = minmod3(e0 - em, rk.kc * (ep - em), ep - e0);
    const float mn = minmod3(n0 - nm, rk.kc * (np - nm), np - n0);
    const float mt = minmod3(t0 - tm, rk.kc * (tp - tm), tp - t0);
    // explicit fused multiply-adds: theta/2 is not a power of two, so a
    // multiply and an add would round differently from one fused operation,
    // and the compiler's choice between the two may differ between kernel
    // instances (strip heights), which must give the same bits
    const float lo_e = fmaf(-rk.hth, me, e0), hi_e = fmaf(rk.hth, me, e0);
    const bool fix_hi = hi_e < -Dhi, fix_lo = !fix_hi && lo_e < -Dlo;
    lo.e = fix_hi ? 2.f * e0 + Dhi : (fix_lo ? -Dlo : lo_e);
    hi.e = fix_hi ? -Dhi : (fix_lo ? 2.f * e0 + Dlo : hi_e);
    lo.n = fmaf(-rk.hth, mn, n0);
    hi.n = fmaf(rk.hth, mn, n0);
    lo.t = fmaf(-rk.hth, mt, t0);
    hi.t = fmaf(rk.hth, mt, t0);
}

// Desingularized velocity sqrt(2) h m / sqrt(h^4 + max(h^4, eps)).
__device__ __forceinline__ float desing(float h, float m, float eps) {
    float h2 = h * h, h4 = h2 * h2;
    return 1.41421356237f * h * m * frsq(h4 + fmaxf(h4, eps));
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
    const float hL = fmaxf(L.e + Df, 0.f), hR = fmaxf(R.e + Df, 0.f);
    const float hL2 = hL * hL, hL4 = hL2 * hL2, hR2 = hR * hR, hR4 = hR2 * hR2;
    // eq. (14): u = m * sqrt(2) h / sqrt(h^4 + max(h^4, eps)), one factor per side
    const float fL = 1.41421356237f * hL * frsq(hL4 + fmaxf(hL4, eps));
    const float fR = 1.41421356237f * hR * frsq(hR4 + fmaxf(hR4, eps));
    const float uL = fL * L.n, vL = fL * L.t, uR = fR * R.n, vR = fR * R.t;
    const float nL = hL * uL, tL = hL * vL, nR = hR * uR, tR = hR * vR;
    const float cL = fsqrt(g * hL), cR = fsqrt(g * hR);
    const float ap = fmaxf(fmaxf(uL + cL, uR + cR), 0.f);
    const float am = fminf(fminf(uL - cL, uR - cR), 0.f);
    const float eL = hL > 0.f ? L.e : -Df, eR = hR > 0.f ? R.e : -Df;
    const float pL = 0.5f * g * eL * (eL + 2.f * Df), pR = 0.5f * g * eR * (eR + 2.f * Df);
    const bool dry = ap - am <= 1e-10f;
    const float inv = frcp(dry ? 1.f : ap - am), apam = ap * am * inv;
    const float m = (ap * nL - am * nR) * inv + apam * (R.e - L.e);
    const float n = (ap * (nL * uL + pL) - am * (nR * uR + pR)) * inv + apam * (nR - nL);
    const float t = (ap * (nL * vL) - am * (nR * vR)) * inv + apam * (tR - tL);
    H0 = dry ? 0.f : m;
    H1 = dry ? -0.5f * g * Df * Df : n;
    H2 = dry ? 0.f : t;
}

// Row/column system coefficients of eq. 23 for one cell, from the cell's
// still-water depth d and the difference dd = d_{+1} - d_{-1} of its two
// neighbours along the direction (d_x = dd / (2 h)).  With the spacing h:
// alpha = (B + 1/3) d^2 / h^2 and beta = d d_x / (6 h) = d dd / (12 h^2), and
// A = beta - alpha, B = 1 + 2 alpha, C = -beta - alpha.  The constant
// factors come premultiplied: kal = (B + 1/3) / h^2, kbe = 1 / (12 h^2).
struct TriK { float kal, kbe; };
__device__ __forceinline__ TriK tri_k(float Bd, float rh) { return {(Bd + 1.f / 3.f) * rh * rh, rh * rh * (1.f / 12.f)}; }
__device__ __forceinline__ void tri_coef_bsnq(TriK k, float dep, float dd, float &A, float &B, float &C) {
    const float al = k.kal * (dep * dep);
    const float be = k.kbe * (dep * dd);
    A = be - al;
    B = 1.f + 2.f * al;
    C = -be - al;
}
__device__ __forceinline__ void tri_coef(const Dom &d, TriK k, float dep, float dd, float &A, float &B,
                                         float &C) {
    if (d.model == NLSW) {
        A = 0.f;
        B = 1.f;
        C = 0.f;
        return;
    }
    tri_coef_bsnq(k, dep, dd, A, B, C);
}

__device__ __forceinline__ float sponge_gamma(float dist, float Ls) {
    return dist >= Ls ? 1.f : 0.5f * (1.f + cosf(3.14159265358979f * (Ls - dist) / Ls));
}
// A partially reflective layer damps by gamma^s (s = 1: the layer of eq. 30).
__device__ __forceinline__ float sponge_factor(float gamma, float s) {
    return s == 1.f ? gamma : s == 0.f ? 1.f : powf(gamma, s);
}

}  // namespace ws
