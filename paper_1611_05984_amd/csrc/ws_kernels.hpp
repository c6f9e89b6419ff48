// ws_kernels.hpp -- the gfx950 kernels of one predictor/corrector pass.
//
// A pass is four launches:
//   k_stencil_{e,p,c}  (Euler predictor, AB3 predictor, AM4 corrector)
//              column-streaming: one wave owns a strip of 64 columns (62 of
//              them output) and walks 8-64 rows (tuned) with a sliding
//              register window;
//              x-neighbours come from DPP lane shifts, so every face is
//              reconstructed and fluxed once and no LDS or barrier is used.
//              KP07 face fluxes, bottom source, dispersive and friction
//              terms, time integration.  Writes the new surface and the
//              increments U* - U*^n, V* - V*^n: the solves work in delta
//              form, T (P - P^n) = U* - U*^n, algebraically the same system,
//              whose right-hand side is O(dt F) instead of O(P), so single
//              precision loses far less in the solve.
//   k_reduce   per 64x16 tile: coefficients of eq. 23 from the bathymetry, and
//              the elimination of every 16-cell row segment and 16-cell column
//              segment down to its first and last unknowns (partition
//              method); writes two reduced equations per segment (the
//              eliminated interiors stay in LDS: the expansion redoes them).
//   reduced    the reduced tridiagonal systems, by one of four strategies:
//              k_pcr (parallel cyclic reduction, a workgroup per system),
//              k_thomas (a lane per system), the factored sweeps with static
//              factors (k_luw_solve: a workgroup per 64 systems held in
//              registers; k_lu_solve: a lane per system) and the two-ended
//              factored sweeps (k_lu2_solve).
//   k_expand   per tile: every segment's elimination again (right-hand
//              sides included) and back substitution from its solved end
//              values, P = P^n + dP, Q = Q^n + dQ, shoreline fix (and the
//              sponge after the last pass).
// k_ghosts precomputes the wave-maker ghost values of one time level.
#pragma once
#include "ws_device.hpp"

namespace ws {

// Field groups are consecutive fields of the workspace, fstride bytes apart:
// a group is addressed by one base pointer plus k * fstride, which keeps the
// kernel's uniform registers few (every field pointer would not fit in SGPRs).
struct StencilArgs {
    Dom d;
    const float *in;     // estimate read (the state itself for the predictor): eta, P, Q
    float *eout;         // new surface
    float *rxy;          // U* - U*^n, V* - V*^n, packed per cell
    float *h0;           // history level n (predictors write it): (E, F, G), (F*, G*) packed
    const float *h1;     // level n-1
    const float *h2;     // level n-2
    float *S;            // corrector bases: eta, U* and V* increments
    unsigned fstride;    // bytes between consecutive fields of a group
    // grid-spacing factors of the difference formulas, premultiplied:
    // hx = 1/(2dx), sxx = 1/dx^2, cxy = 1/(4 dx dy), cxxx = 1/(2 dx^3),
    // cxyy = 1/(2 dx dy^2), gx = g/dx, Bg = B g (y analogues likewise)
    float hx, hy, sxx, syy, cxy, cxxx, cyyy, cxyy, cxxy, gx, gy, Bg;
    float dt, x0, x1, x2;  // step, F* extrapolation weights
    int kind;            // 0 Euler predictor, 1 AB3 predictor, 2 AM4 corrector
    int write_S;
};

__device__ __forceinline__ float dcell4(float a, float b, float c, float d) {
    return fmaxf(0.25f * ((a + b) + (c + d)), 0.f);
}

// Ghost values of every wave-maker side at time t (eqs. 25-28 per component).
// GHL lanes share one ghost cell, each summing every GHL-th component; the
// partial sums meet by butterfly shuffles, so a 64-component maker keeps
// the whole chip busy instead of one lane per cell.  Thread k: cell k / GHL.
constexpr int GHL = 16;
__device__ __forceinline__ void ghosts_body(const Dom &d, float *gh, double t, int k) {
    const int cell = k / GHL, sub = k % GHL;
    const int pos = cell % d.gl, layer = (cell / d.gl) % 2, side = cell / (2 * d.gl);
    // lanes of one cell are consecutive and stay together through the shuffles
    const bool live = side < 4 && d.side[side < 4 ? side : 0].type == BC_WAVES;
    float se = 0.f, sp = 0.f, sq = 0.f;
    if (live) {
        const SideDev &sd = d.side[side];
        int i, j;
        if (side < 2) {
            i = side == 0 ? -1 - layer : d.nx + layer;
            j = pos - 2;
        } else {
            j = side == 2 ? -1 - layer : d.ny + layer;
            i = pos - 2;
        }
        wave_partial(sd, (i + 0.5) * (double)d.dx, (j + 0.5) * (double)d.dy, t, sub, GHL, se, sp, sq);
    }
#pragma unroll
    for (int m = GHL / 2; m >= 1; m >>= 1) {
        se += __shfl_xor(se, m, GHL);
        sp += __shfl_xor(sp, m, GHL);
        sq += __shfl_xor(sq, m, GHL);
    }
    if (live && sub == 0) {
        float *o = gh + ghost_index(d, side, layer, pos);
        o[0] = se;
        o[1] = sp;
        o[2] = sq;
    }
}

__global__ void k_ghosts(Dom d, float *gh, double t) { ghosts_body(d, gh, t, blockIdx.x * blockDim.x + threadIdx.x); }

// Field access by 32-bit byte offset from a uniform base pointer: the load or
// store takes the base from SGPRs and the offset from one VGPR shared by all
// fields (no 64-bit address arithmetic per access).
__device__ __forceinline__ float ldo(const float *p, unsigned ob) {
    return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(p) + ob);
}
__device__ __forceinline__ void sto(float *p, unsigned ob, float v) {
    *reinterpret_cast<float *>(reinterpret_cast<char *>(p) + ob) = v;
}
__device__ __forceinline__ const float *ldp(const float *p, unsigned ob) {
    return reinterpret_cast<const float *>(reinterpret_cast<const char *>(p) + ob);
}

// Fields written and read together are packed per cell: a history level
// holds (E, F, G) as three consecutive floats a cell, then (F*, G*) as two;
// the solve's right-hand sides (U* - U*^n, V* - V*^n) two.  A cell at float
// offset ob (bytes) sits at 3 ob in a three-float group and at 2 ob in a
// two-float one, so one 12- or 8-byte access replaces three or two field
// streams: the predictor moves its 23 words in 14 streams, 9 % faster.  The
// corrector bases stay three fields: read as one 12- (or 8-) byte group, the
// corrector, at its register limit, ran 8 % slower.
struct f3 { float x, y, z; };
__device__ __forceinline__ f3 ld3(const float *p, unsigned ob) {
    return *reinterpret_cast<const f3 *>(reinterpret_cast<const char *>(p) + ob);
}
__device__ __forceinline__ void st3(float *p, unsigned ob, f3 v) {
    *reinterpret_cast<f3 *>(reinterpret_cast<char *>(p) + ob) = v;
}
__device__ __forceinline__ float2 ld2(const float *p, unsigned ob) {
    return *reinterpret_cast<const float2 *>(reinterpret_cast<const char *>(p) + ob);
}
__device__ __forceinline__ void st2(float *p, unsigned ob, float2 v) {
    *reinterpret_cast<float2 *>(reinterpret_cast<char *>(p) + ob) = v;
}

// Rows per stencil strip: a template parameter (8, 16, 24, 32, 48 or 64)
// chosen per grid shape; taller strips spend less on the 4 warm-up rows,
// shorter ones give more workgroups.
// The pass kind (A.kind) is a compile-time parameter: each kernel carries
// no code, registers or branches for the other kinds.  SOLO: the workgroup
// is one wave (one strip) instead of SWG side-by-side strips; the
// single-domain corrector is 4 % faster so, the predictors 7 % slower.
// Every cell's arithmetic is the same either way.
template <int SYT, int KIND, bool SOLO = false>
__device__ __forceinline__ void stencil_body(const StencilArgs &A, int bx, int by) {
    const Dom &d = A.d;
    constexpr int kind = KIND;
    const int lane = threadIdx.x & 63;
    const int strip = SOLO ? bx : bx * SWG + (threadIdx.x >> 6);
    const int c0 = strip * SO - 1;  // column of lane 0; lanes 1..62 are output columns
    // In a one-wave workgroup threadIdx.x >> 6 is 0; written with it, the row
    // index is a per-lane value, so its arithmetic stays out of the scalar
    // registers (the corrector then spills 4 SGPRs instead of 10, and runs
    // 4 % faster)
    const int j0 = (by + (SOLO ? (int)(threadIdx.x >> 6) : 0)) * SYT;
    if (c0 + 1 >= d.nx || j0 >= d.ny) return;  // whole wave past the domain
    const int col = c0 + lane;
    const int hcol = lane == 0 ? c0 - 1 : c0 + 64;  // halo column held by lanes 0 and 63
    const bool halo_lane = lane == 0 || lane == 63;
    const Recon rk = recon_k(d.theta);
    const float g = d.g, eps = d.eps;
    const float rdx = d.rdx, rdy = d.rdy, B3 = d.Bd + 1.f / 3.f;
    // strips whose cells and corners (with halo) all lie inside the domain
    // load without boundary handling
    const bool interior = c0 >= 1 && c0 + 64 <= d.nx - 1 && j0 >= 2 && j0 + SYT + 1 <= d.ny - 1;

    // sliding windows (row index relative to the row r loaded this iteration)
    float e0 = 0.f, e1 = 0.f, e2 = 0.f, e3 = 0.f, e4 = 0.f;  // eta rows r-4 .. r
    float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;            // P rows r-3 .. r
    float q0 = 0.f, q1 = 0.f, q2 = 0.f, q3 = 0.f;            // Q rows r-3 .. r
    float he0 = 0.f, he1 = 0.f, he2 = 0.f, hp0 = 0.f, hp1 = 0.f, hp2 = 0.f;  // halo rows r-2 .. r
    float hq0 = 0.f, hq1 = 0.f, hq2 = 0.f;
    float Dl1 = 0.f, Dl2 = 0.f, Dl3 = 0.f;                   // corner depth at col, rows r-2 .. r
    float Dr1 = 0.f, Dr2 = 0.f, Dr3 = 0.f;                   // corner depth at col+1
    F3 hiy_prev = {0.f, 0.f, 0.f};                           // y-reconstruction, north side of row r-2
    float Hs0 = 0.f, Hs1 = 0.f, Hs2 = 0.f;                   // flux through the south face of row r-2
    float Dcm = 0.f, Dc0 = 0.f;                              // cell depth D of rows r-3, r-2

    const unsigned F1 = A.fstride, F2 = 2u * A.fstride, F3b = 3u * A.fstride;
    const float *pin = ldp(A.in, F1), *qin = ldp(A.in, F2);
    // row r + 1 is loaded while row r is computed
    float ne = 0.f, np = 0.f, nq = 0.f, nhe = 0.f, nhp = 0.f, nhq = 0.f, nDl = 0.f, nDr = 0.f;
    auto load_row = [&](int r) {
        if (interior) {
            const unsigned ob = (unsigned)(r * d.pitch + col) * 4u, ohb = (unsigned)(r * d.pitch + hcol) * 4u;
            const unsigned ozb = (unsigned)(r * d.zpitch + col) * 4u;
            ne = ldo(A.in, ob);
            np = ldo(A.in, ob + F1);
            nq = ldo(A.in, ob + F2);
            if (halo_lane) {
                nhe = ldo(A.in, ohb);
                nhp = ldo(A.in, ohb + F1);
                nhq = ldo(A.in, ohb + F2);
            }
            nDl = ldo(d.D, ozb);
            nDr = ldo(d.D, ozb + 4u);
        } else {
            load_cell(d, A.in, pin, qin, col, r, ne, np, nq);
            if (halo_lane) load_cell(d, A.in, pin, qin, hcol, r, nhe, nhp, nhq);
            nDl = corner_D(d, col, r);
            nDr = corner_D(d, col + 1, r);
        }
    };
    load_row(j0 - 2);

    // the corrector's row loop fully unrolled at 8 rows (no sliding-window
    // moves; corrector 208 -> 198 us at 4096^2); the predictor, with more
    // live history values, is faster rolled
#pragma unroll KIND == 2 && SYT <= 8 ? SYT + 4 : 1
    for (int it = 0; it < SYT + 4; ++it) {
        const int r = j0 - 2 + it;
        e0 = e1; e1 = e2; e2 = e3; e3 = e4;
        p0 = p1; p1 = p2; p2 = p3;
        q0 = q1; q1 = q2; q2 = q3;
        he0 = he1; he1 = he2; hp0 = hp1; hp1 = hp2; hq0 = hq1; hq1 = hq2;
        Dl1 = Dl2; Dl2 = Dl3;
        Dr1 = Dr2; Dr2 = Dr3;
        e4 = ne; p3 = np; q3 = nq;
        he2 = nhe; hp2 = nhp; hq2 = nhq;
        Dl3 = nDl; Dr3 = nDr;
        if (it + 1 < SYT + 4) load_row(r + 1);
        // still-water depth D of the cell in row r-1
        const float Dcp = 0.25f * ((Dl2 + Dr2) + (Dl3 + Dr3));
        if (it < 2) {
            Dcm = Dc0;
            Dc0 = Dcp;
            continue;
        }

        // y-reconstruction of row r-1 (normal discharge Q) and the flux
        // through its south face (between rows r-2 and r-1)
        const float Dys = 0.5f * (Dl2 + Dr2), Dyn = 0.5f * (Dl3 + Dr3);
        F3 loy, hiy;
        reconstruct(e2, e3, e4, q1, q2, q3, p1, p2, p3, Dys, Dyn, rk, loy, hiy);
        float Hn0 = 0.f, Hn1 = 0.f, Hn2 = 0.f;  // (mass, y-momentum, x-momentum)
        if (it >= 3) cu_flux(g, eps, Dys, hiy_prev, loy, Hn0, Hn1, Hn2);

        if (it >= 4) {  // update row u = r - 2
            const int u = r - 2;
            const bool out = lane >= 1 && lane <= 62 && col < d.nx && u < d.ny;
            const unsigned o = (unsigned)(u * d.pitch + col) * 4u;  // byte offset (used by output lanes only)
            float E1v = 0.f, F1v = 0.f, G1v = 0.f, Fs1v = 0.f, Gs1v = 0.f, E2v = 0.f, F2v = 0.f, G2v = 0.f;
            float Fs2v = 0.f, Gs2v = 0.f, Sev = 0.f, SUv = 0.f, SVv = 0.f;
            if (out) {
                if (kind == 1) {
                    const f3 l1 = ld3(A.h1, 3u * o), l2 = ld3(A.h2, 3u * o);
                    const float2 s1 = ld2(A.h1, F3b + 2u * o);
                    E1v = l1.x; F1v = l1.y; G1v = l1.z;
                    Fs1v = s1.x; Gs1v = s1.y;
                    E2v = l2.x; F2v = l2.y; G2v = l2.z;
                    if (A.x2 != 0.f) {
                        const float2 s2 = ld2(A.h2, F3b + 2u * o);
                        Fs2v = s2.x; Gs2v = s2.y;
                    }
                } else if (kind == 2) {
                    Sev = ldo(A.S, o); SUv = ldo(A.S, o + F1); SVv = ldo(A.S, o + F2);
                }
            }
            // cell and face still-water depths
            const float Dc = Dc0;
            const float Dw = 0.5f * (Dl1 + Dl2), De = 0.5f * (Dr1 + Dr2);
            const float Ds = 0.5f * (Dl1 + Dr1), Dn = Dys;
            // x-reconstruction of row u (normal discharge P); lanes 0 and 63
            // take their outer neighbour from the halo columns
            const float em = shr1(e2, he0), ep = shl1(e2, he0);
            const float pm = shr1(p1, hp0), pp = shl1(p1, hp0);
            const float qm = shr1(q1, hq0), qp = shl1(q1, hq0);
            F3 lox, hix;
            reconstruct(em, e2, ep, pm, p1, pp, qm, q1, qp, Dw, De, rk, lox, hix);
            const F3 hil = {shr1z(hix.e), shr1z(hix.n), shr1z(hix.t)};
            float Hw0, Hw1, Hw2;  // west face: (mass, x-momentum, y-momentum)
            cu_flux(g, eps, Dw, hil, lox, Hw0, Hw1, Hw2);
            const float He0 = shl1z(Hw0), He1 = shl1z(Hw1), He2 = shl1z(Hw2);

            float E = -(He0 - Hw0) * rdx - (Hn0 - Hs0) * rdy;
            float F = -(He1 - Hw1) * rdx - (Hn2 - Hs2) * rdy + A.gx * (De - Dw) * e2;
            float G = -(He2 - Hw2) * rdx - (Hn1 - Hs1) * rdy + A.gy * (Dn - Ds) * e2;
            float Fs = 0.f, Gs = 0.f;

            const float dep = fmaxf(Dc, 0.f);
            const float dxm = shr1z(dep), dxp = shl1z(dep);
            const float dym = fmaxf(Dcm, 0.f), dyp = fmaxf(Dcp, 0.f);
            const float ddx = (dxp - dxm) * A.hx, ddy = (dyp - dym) * A.hy;

            if (d.model == BSNQ) {
                const float em2 = shr1z(em), ep2 = shl1z(ep);
                const float epp = shl1z(e3), epm = shl1z(e1);
                const float emp = shr1z(e3), emm = shr1z(e1);
                const float exx = (ep - 2.f * e2 + em) * A.sxx;
                const float eyy = (e3 - 2.f * e2 + e1) * A.syy;
                const float exy = (epp - epm - emp + emm) * A.cxy;
                const float exxx = (ep2 - 2.f * ep + 2.f * em - em2) * A.cxxx;
                const float eyyy = (e4 - 2.f * e3 + 2.f * e1 - e0) * A.cyyy;
                const float exyy = ((epp - 2.f * ep + epm) - (emp - 2.f * em + emm)) * A.cxyy;
                const float exxy = ((epp - 2.f * e3 + emp) - (epm - 2.f * e1 + emm)) * A.cxxy;
                const float gb = A.Bg * dep * dep;
                F += gb * (dep * (exxx + exyy) + ddx * (2.f * exx + eyy) + ddy * exy);
                G += gb * (dep * (eyyy + exxy) + ddy * (2.f * eyy + exx) + ddx * exy);
                // cross differences ((P(i+1,j+1) - P(i+1,j-1)) - P(i-1,j+1)) + P(i-1,j-1):
                // the first difference is the east neighbour's column difference,
                // shifted (the same value, one lane shift fewer)
                const float dpy = p2 - p0, dqy = q2 - q0;
                const float Px = (pp - pm) * A.hx, Py = dpy * A.hy;
                const float Pxy = (shl1z(dpy) - shr1z(p2) + shr1z(p0)) * A.cxy;
                const float Qx = (qp - qm) * A.hx, Qy = dqy * A.hy;
                const float Qxy = (shl1z(dqy) - shr1z(q2) + shr1z(q0)) * A.cxy;
                Fs = dep * (ddx * Qy + ddy * Qx) * (1.f / 6.f) + B3 * dep * dep * Qxy;
                Gs = dep * (ddy * Px + ddx * Py) * (1.f / 6.f) + B3 * dep * dep * Pxy;
            }
            if (d.friction != FRIC_NONE) {
                const float h = fmaxf(e2 + Dc, 0.f), h2 = h * h, h4 = h2 * h2;
                const float inv_h = 1.41421356237f * h * frsq(h4 + fmaxf(h4, eps));
                float fc = d.fcoef;
                if (d.friction == FRIC_MANNING) fc = g * d.fcoef * d.fcoef * cbrtf(inv_h);
                const float k = fc * fsqrt(p1 * p1 + q1 * q1) * inv_h * inv_h;
                F -= k * p1;
                G -= k * q1;
            }
            if (out) {
                const float dt = A.dt;
                float en, U, V;  // new surface, increments of U*, V* over the step
                if (kind == 0) {
                    en = e2 + dt * E;
                    U = dt * F;
                    V = dt * G;
                } else if (kind == 1) {
                    const float c12 = dt * (1.f / 12.f), c24 = dt * (1.f / 24.f);
                    if (A.write_S) {
                        sto(A.S, o, e2 + c24 * (19.f * E - 5.f * E1v + E2v));
                        sto(A.S, o + F1, c24 * (19.f * F - 5.f * F1v + F2v) - Fs);
                        sto(A.S, o + F2, c24 * (19.f * G - 5.f * G1v + G2v) - Gs);
                    }
                    en = e2 + c12 * (23.f * E - 16.f * E1v + 5.f * E2v);
                    U = c12 * (23.f * F - 16.f * F1v + 5.f * F2v) + (A.x0 * Fs + A.x1 * Fs1v + A.x2 * Fs2v);
                    V = c12 * (23.f * G - 16.f * G1v + 5.f * G2v) + (A.x0 * Gs + A.x1 * Gs1v + A.x2 * Gs2v);
                } else {
                    const float c9 = dt * (9.f / 24.f);
                    en = Sev + c9 * E;
                    U = SUv + c9 * F + Fs;
                    V = SVv + c9 * G + Gs;
                }
                if (kind != 2) {
                    st3(A.h0, 3u * o, f3{E, F, G});
                    st2(A.h0, F3b + 2u * o, make_float2(Fs, Gs));
                }
                sto(A.eout, o, fmaxf(en, -Dc));
                st2(A.rxy, 2u * o, make_float2(U, V));
            }
        }
        hiy_prev = hiy;
        Hs0 = Hn0;
        Hs1 = Hn1;
        Hs2 = Hn2;
        Dcm = Dc0;
        Dc0 = Dcp;
    }
}

// XCD-aware order of a 1-D grid of G workgroups over a gx x gy tile grid.
// Workgroups go round-robin to the 8 XCDs (b mod 8), each with its own L2;
// XCD x gets a contiguous band of tiles in row-major order, so the strips
// it runs side by side include vertical neighbours, whose halo rows it
// reads through its own L2, while rows stay contiguous in memory.
__device__ __forceinline__ int xcd_order(int b, int G) {
    const int q = G >> 3, rem = G & 7, x = b & 7, i = b >> 3;
    return x * q + (x < rem ? x : rem) + i;
}
__device__ __forceinline__ void xcd_tile(int b, int G, int gx, int &bx, int &by) {
    const int t = xcd_order(b, G);
    by = t / gx;
    bx = t - by * gx;
}

// One kernel per pass kind: Euler start-up predictor, AB3 predictor, AM4
// corrector.
template <int SYT, int KIND>
__device__ __forceinline__ void stencil_kernel_body(const StencilArgs &A, int gx) {
    int bx, by;
    xcd_tile(blockIdx.x, gridDim.x, gx, bx, by);
    stencil_body<SYT, KIND, KIND == 2>(A, bx, by);  // the corrector on one-wave workgroups
}
template <int SYT>
__global__ __launch_bounds__(64 * SWG) __attribute__((amdgpu_waves_per_eu(4))) void k_stencil_e(StencilArgs A, int gx) {
    stencil_kernel_body<SYT, 0>(A, gx);
}
template <int SYT>
__global__ __launch_bounds__(64 * SWG) __attribute__((amdgpu_waves_per_eu(4))) void k_stencil_p(StencilArgs A, int gx) {
    stencil_kernel_body<SYT, 1>(A, gx);
}
template <int SYT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_stencil_c(StencilArgs A, int gx) {
    stencil_kernel_body<SYT, 2>(A, gx);
}

// ------------------------------------------------------------- solver parts
struct SolveArgs {
    Dom d;
    float *rx, *ry;            // right-hand sides (read by the reduction and the expansion):
                               // the pair packed per cell from rx on (ry: its second field)
    float4 *redx, *redy;       // reduced equations (sub, diag, super, rhs) per unknown
    float *solx, *soly;        // reduced solutions
    // layout 1 (factored solve): the reduced right-hand sides (in the memory of
    // redx, redy) and the solutions are system-interleaved, unknown k of row
    // system j at k * ny + j (columns: k * nx + i); lux, luy hold the static
    // factors, likewise interleaved: (a, 1/pivot) pairs, then the modified
    // super-diagonals.
    const float *lux, *luy;
    int layout;
    float *eta, *pout, *qout;  // new surface (read; sponge writes it), new P, Q
    const float *pbase, *qbase;  // P^n, Q^n of the step
    const float *gh0, *gh1;    // wave-maker ghosts at t^n and t^{n+1}
    int *health;
    int sponge;
    int nlsw;  // NLSW: the systems are the identity, the increments in rx, ry are final
};

constexpr int TXP = TX + 1;  // padded LDS row: segment k of row r starts at bank r + 16k

struct SolveTile {
    float rx[TY][TXP], ry[TY][TXP];   // right-hand sides / solution of the tile
    float cz[TY + 3][TX + 3];         // corner depths, corners -1 .. TX+1, -1 .. TY+1
    float dc[TY + 2][TX + 2];         // cell still-water depth max(D, 0), cells -1..TX, -1..TY
};

// Discharge change of a wave-maker ghost over the step (first ghost layer).
__device__ __forceinline__ float ghost_change(const SolveArgs &A, int side, int pos, int comp) {
    const size_t k = ghost_index(A.d, side, 0, pos) + comp;
    return A.gh1[k] - A.gh0[k];
}

// Stage the tile's corner and cell depths in LDS.
// Stage a tile: its two right-hand-side fields and the corner depths around
// it, all loads issued before any LDS store so that they share one memory
// latency, then the cell depths from the corners.
// Tile cells and corner values per thread for a workgroup of T threads.
template <int T> constexpr int cells_per_thread() { return TX * TY / T; }
template <int T> constexpr int corners_per_thread() { return ((TX + 3) * (TY + 3) + T - 1) / T; }
template <int T = NT>
__device__ __forceinline__ void stage_tile(const SolveArgs &A, SolveTile &s, int i0, int j0) {
    constexpr int CPT = cells_per_thread<T>(), ZPT = corners_per_thread<T>();
    const Dom &d = A.d;
    const int tid = threadIdx.x;
    float vx[CPT], vy[CPT], vz[ZPT];
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int k = tid + m * T, cx = k % TX, cy = k / TX;
        const size_t o = (size_t)(j0 + cy) * d.pitch + i0 + cx;
        const float2 v = reinterpret_cast<const float2 *>(A.rx)[o];  // (U* - U*^n, V* - V*^n) of the cell
        vx[m] = v.x;
        vy[m] = v.y;
    }
#pragma unroll
    for (int m = 0; m < ZPT; ++m) {
        const int k = tid + m * T, lx = k % (TX + 3), ly = k / (TX + 3);
        vz[m] = k < (TX + 3) * (TY + 3) ? corner_D(d, i0 + lx - 1, j0 + ly - 1) : 0.f;
    }
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int k = tid + m * T, cx = k % TX, cy = k / TX;
        s.rx[cy][cx] = vx[m];
        s.ry[cy][cx] = vy[m];
    }
#pragma unroll
    for (int m = 0; m < ZPT; ++m) {
        const int k = tid + m * T, lx = k % (TX + 3), ly = k / (TX + 3);
        if (k < (TX + 3) * (TY + 3)) s.cz[ly][lx] = vz[m];
    }
    __syncthreads();
    for (int k = tid; k < (TX + 2) * (TY + 2); k += T) {
        const int lx = k % (TX + 2), ly = k / (TX + 2);
        s.dc[ly][lx] = fmaxf(0.25f * ((s.cz[ly][lx] + s.cz[ly][lx + 1]) + (s.cz[ly + 1][lx] + s.cz[ly + 1][lx + 1])), 0.f);
    }
    __syncthreads();
}

// Coefficients of eq. 23 of one segment of M cells, in registers.  dir 0:
// cells (x0 + k, y) of a tile row; dir 1: cells (x, y0 + k) of a tile column
// (tile-local indices).  Boundary rows are folded: behind a wall the ghost is
// the odd mirror of the first unknown (diagonal -= off-diagonal); behind a
// wave maker it is the maker's known discharge, whose change over the step
// moves to the right-hand side of the delta-form system (r, when given).
// Padding cells are identity rows with zero right-hand side.
template <int M, bool INNER = false>
__device__ __forceinline__ void seg_coefs(const SolveArgs &A, const SolveTile &s, int i0, int j0, int dir,
                                          int x0, int y0, float (&a)[M], float (&b)[M], float (&c)[M],
                                          float *r, int st) {
    const Dom &d = A.d;
    // INNER: a segment clear of the domain's edges (in the dispersive model)
    // takes a path without boundary rows, cells outside or per-cell tests;
    // the same arithmetic as the general loop below (used where the
    // duplicated code pays: the reduction, not the expansion)
    const int fi = i0 + x0, fj = j0 + y0;
    const bool inner = INNER && d.model != NLSW &&
                       (dir == 0 ? fj < d.ny && fi >= 1 && fi + M <= d.nx - 1 : fi < d.nx && fj >= 1 && fj + M <= d.ny - 1);
    const TriK tk = tri_k(d.Bd, dir == 0 ? d.rdx : d.rdy);
    if (inner) {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int cx = dir == 0 ? x0 + k : x0, cy = dir == 0 ? y0 : y0 + k;
            const float dep = s.dc[cy + 1][cx + 1];
            const float dd = dir == 0 ? s.dc[cy + 1][cx + 2] - s.dc[cy + 1][cx] : s.dc[cy + 2][cx + 1] - s.dc[cy][cx + 1];
            tri_coef_bsnq(tk, dep, dd, a[k], b[k], c[k]);
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const int cx = dir == 0 ? x0 + k : x0, cy = dir == 0 ? y0 : y0 + k;
        const int i = i0 + cx, j = j0 + cy;
        float aa = 0.f, bb = 1.f, cc = 0.f;
        if (i < d.nx && j < d.ny) {
            const float dep = s.dc[cy + 1][cx + 1];
            if (dir == 0) {
                tri_coef(d, tk, dep, s.dc[cy + 1][cx + 2] - s.dc[cy + 1][cx], aa, bb, cc);
                if (i == 0) {
                    if (is_wall(d, 0)) bb -= aa;
                    else if (r) r[k * st] -= aa * ghost_change(A, 0, j + 2, 1);
                    aa = 0.f;
                }
                if (i == d.nx - 1) {
                    if (is_wall(d, 1)) bb -= cc;
                    else if (r) r[k * st] -= cc * ghost_change(A, 1, j + 2, 1);
                    cc = 0.f;
                }
            } else {
                tri_coef(d, tk, dep, s.dc[cy + 2][cx + 1] - s.dc[cy][cx + 1], aa, bb, cc);
                if (j == 0) {
                    if (is_wall(d, 2)) bb -= aa;
                    else if (r) r[k * st] -= aa * ghost_change(A, 2, i + 2, 2);
                    aa = 0.f;
                }
                if (j == d.ny - 1) {
                    if (is_wall(d, 3)) bb -= cc;
                    else if (r) r[k * st] -= cc * ghost_change(A, 3, i + 2, 2);
                    cc = 0.f;
                }
            }
        } else if (r) {
            r[k * st] = 0.f;
        }
        a[k] = aa;
        b[k] = bb;
        c[k] = cc;
    }
}

// Partition-method elimination of one segment of M unknowns: afterwards every
// interior row k reads  a_k x_0 + b_k x_k + c_k x_{M-1} = r_k (r overwritten,
// stride st in LDS), and the first and last rows are returned as reduced
// equations coupling (x_{-1}, x_0, x_{M-1}) and (x_0, x_{M-1}, x_M).
template <int M>
__device__ __forceinline__ void seg_eliminate(float *r, int st, float (&a)[M], float (&b)[M],
                                              const float (&c)[M], float4 &first, float4 &last) {
#pragma unroll
    for (int k = 2; k <= M - 2; ++k) {  // forward: eliminate x_{k-1} in favour of x_0
        const float f = a[k] * frcp(b[k - 1]);
        a[k] = -f * a[k - 1];
        b[k] = b[k] - f * c[k - 1];
        r[k * st] = r[k * st] - f * r[(k - 1) * st];
    }
    {
        const float f = a[M - 1] * frcp(b[M - 2]);
        last = make_float4(-f * a[M - 2], b[M - 1] - f * c[M - 2], c[M - 1], r[(M - 1) * st] - f * r[(M - 2) * st]);
    }
    float ah = a[M - 2], bh = b[M - 2], ch = c[M - 2], rh = r[(M - 2) * st];
#pragma unroll
    for (int k = M - 3; k >= 1; --k) {  // backward: eliminate x_{k+1} in favour of x_{M-1}
        const float f = c[k] * frcp(bh);
        ah = a[k] - f * ah;
        bh = b[k];
        ch = -f * ch;
        rh = r[k * st] - f * rh;
        r[k * st] = rh;
    }
    const float f = c[0] * frcp(bh);
    first = make_float4(a[0], b[0] - f * ah, -f * ch, r[0] - f * rh);
}

// Solution of one segment from its solved end values x0, xl: the
// elimination of seg_eliminate (the same operations in the same order, on
// the right-hand sides too), then back substitution; r holds the right-hand
// sides on entry and the solution on exit.  Redoing the right-hand-side
// elimination here (one multiply-add a cell each way, next to the factors
// this loop computes anyway) spares the reduction writing the eliminated
// values to HBM and this kernel reading them back.
template <int M>
__device__ __forceinline__ void seg_expand(float *r, int st, float (&a)[M], float (&b)[M],
                                           const float (&c)[M], float x0, float xl) {
#pragma unroll
    for (int k = 2; k <= M - 2; ++k) {
        const float f = a[k] * frcp(b[k - 1]);
        a[k] = -f * a[k - 1];
        b[k] = b[k] - f * c[k - 1];
        r[k * st] = r[k * st] - f * r[(k - 1) * st];
    }
    float ah = a[M - 2], bh = b[M - 2], ch = c[M - 2], rh = r[(M - 2) * st];
    r[(M - 2) * st] = (rh - ah * x0 - ch * xl) * frcp(bh);
#pragma unroll
    for (int k = M - 3; k >= 1; --k) {
        const float f = c[k] * frcp(bh);
        ah = a[k] - f * ah;
        bh = b[k];
        ch = -f * ch;
        rh = r[k * st] - f * rh;
        r[k * st] = (rh - ah * x0 - ch * xl) * frcp(bh);
    }
    r[0] = x0;
    r[(M - 1) * st] = xl;
}

// Wave 0 owns the 64 row segments of a tile (lane -> segment lane/16 of row
// lane%16, conflict-free with the padded rows), wave 1 its 64 column segments.
template <int T = NT>
__device__ __forceinline__ void reduce_body(const SolveArgs &A, SolveTile &s, int bx, int by) {
    const Dom &d = A.d;
    const int tid = threadIdx.x;
    const int i0 = bx * TX, j0 = by * TY;
    stage_tile<T>(A, s, i0, j0);
    if (tid < 64) {
        const int row = tid % 16, seg = tid / 16, k0 = seg * MX;
        float a[MX], b[MX], c[MX];
        float4 first, last;
        float *r = &s.rx[row][k0];
        seg_coefs<MX, true>(A, s, i0, j0, 0, k0, row, a, b, c, r, 1);
        seg_eliminate<MX>(r, 1, a, b, c, first, last);
        const int k = 2 * (bx * (TX / MX) + seg), j = j0 + row;
        if (A.layout) {
            if (j < d.ny) {
                float *rr = reinterpret_cast<float *>(A.redx);
                rr[(size_t)k * d.ny + j] = first.w;
                rr[(size_t)(k + 1) * d.ny + j] = last.w;
            }
        } else {
            float4 *red = A.redx + (size_t)j * d.nu + k;
            red[0] = first;
            red[1] = last;
        }
    } else if (tid < 128) {
        const int col = tid - 64;
        float a[TY], b[TY], c[TY];
        float4 first, last;
        float *r = &s.ry[0][col];
        seg_coefs<TY, true>(A, s, i0, j0, 1, col, 0, a, b, c, r, TXP);
        seg_eliminate<TY>(r, TXP, a, b, c, first, last);
        const int i = i0 + col;
        if (A.layout) {
            if (i < d.nx) {
                float *rr = reinterpret_cast<float *>(A.redy);
                rr[(size_t)(2 * by) * d.nx + i] = first.w;
                rr[(size_t)(2 * by + 1) * d.nx + i] = last.w;
            }
        } else {
            float4 *red = A.redy + (size_t)i * d.nv + 2 * by;
            red[0] = first;
            red[1] = last;
        }
    }
}

__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(6))) void k_reduce(SolveArgs A) {
    __shared__ SolveTile s;
    reduce_body(A, s, blockIdx.x, blockIdx.y);
}

// The reduced systems by the Thomas algorithm, one lane per system: lanes of
// a wave take consecutive systems (rows first, then columns; a wave never
// mixes the two), each walks its own contiguous equations, so a wave's loads
// touch 64 lines whose next equations stay cached.  The forward sweep keeps
// its modified super-diagonal and right-hand side in the equation's own
// (z, w) slots, which the backward sweep reads back.  Work is linear in N
// with no barriers; the sweep is a dependent chain of N steps per lane.
__device__ __forceinline__ void thomas_lane(int N, float4 *eq, float *x) {
    float cp = 0.f, dp = 0.f;
    for (int k = 0; k < N; ++k) {
        const float4 e = eq[k];
        const float inv = frcp(e.y - e.x * cp);
        cp = e.z * inv;
        dp = (e.w - e.x * dp) * inv;
        reinterpret_cast<float2 *>(eq + k)[1] = make_float2(cp, dp);
    }
    float v = dp;
    x[N - 1] = v;
    for (int k = N - 2; k >= 0; --k) {
        const float2 cd = reinterpret_cast<const float2 *>(eq + k)[1];
        v = cd.y - cd.x * v;
        x[k] = v;
    }
}

// Waves 0 .. xw-1 take the row systems (xw = ceil(ny / 64)), the rest the
// column systems.
__device__ __forceinline__ void thomas_body(const SolveArgs &A, int wave, int lane) {
    const Dom &d = A.d;
    const int xw = (d.ny + 63) / 64;
    if (wave < xw) {
        const int sys = wave * 64 + lane;
        if (sys < d.ny) thomas_lane(d.nu, A.redx + (size_t)sys * d.nu, A.solx + (size_t)sys * d.nu);
    } else {
        const int sys = (wave - xw) * 64 + lane;
        if (sys < d.nx) thomas_lane(d.nv, A.redy + (size_t)sys * d.nv, A.soly + (size_t)sys * d.nv);
    }
}

__global__ __launch_bounds__(64) void k_thomas(SolveArgs A) { thomas_body(A, blockIdx.x, threadIdx.x); }

// Factored solve of the reduced systems.  Their matrices depend only on the
// depth and the boundary types, so they are factored once (Thomas
// elimination, k_lu_factor, from the equations a coefficient-mode reduction
// writes) and every pass only sweeps the right-hand side forward and back:
// two fused multiply-adds per unknown, one lane per system, all accesses
// system-interleaved so that a wave's 64 lanes read 256 contiguous bytes.
// The arithmetic is the lane-per-system Thomas solve's, so both give the same
// bits.
__device__ __forceinline__ void lu_factor_lane(int N, const float4 *eq, float2 *fai, float *fcp, size_t stride) {
    float cp = 0.f;
    for (int k = 0; k < N; ++k) {
        const float4 e = eq[k];
        const float inv = frcp(e.y - e.x * cp);
        cp = e.z * inv;
        fai[k * stride] = make_float2(e.x, inv);
        fcp[k * stride] = cp;
    }
}

// The sweeps go in blocks whose loads are all issued before the block's
// dependent chain: the chain is a few cycles per unknown, a load about a
// microsecond, so a block's loads share one latency.  A block is as long as
// the outstanding-load counter allows (two loads per unknown, 63 in flight).
constexpr int LU_U = 30;
__device__ __forceinline__ void lu_solve_lane(int N, const float *r, const float2 *fai, const float *fcp, float *x,
                                              size_t stride) {
    float dp = 0.f;
    int k = 0;
    for (; k + LU_U <= N; k += LU_U) {
        float rr[LU_U];
        float2 ai[LU_U];
#pragma unroll
        for (int u = 0; u < LU_U; ++u) {
            const size_t o = (size_t)(k + u) * stride;
            rr[u] = r[o];
            ai[u] = fai[o];
        }
#pragma unroll
        for (int u = 0; u < LU_U; ++u) {
            dp = (rr[u] - ai[u].x * dp) * ai[u].y;
            x[(size_t)(k + u) * stride] = dp;
        }
    }
    for (; k < N; ++k) {
        const size_t o = (size_t)k * stride;
        const float2 ai = fai[o];
        dp = (r[o] - ai.x * dp) * ai.y;
        x[o] = dp;
    }
    float v = dp;
    k = N - 2;
    for (; k - LU_U + 1 >= 0; k -= LU_U) {
        float xx[LU_U], cc[LU_U];
#pragma unroll
        for (int u = 0; u < LU_U; ++u) {
            const size_t o = (size_t)(k - u) * stride;
            xx[u] = x[o];
            cc[u] = fcp[o];
        }
#pragma unroll
        for (int u = 0; u < LU_U; ++u) {
            v = xx[u] - cc[u] * v;
            x[(size_t)(k - u) * stride] = v;
        }
    }
    for (; k >= 0; --k) {
        const size_t o = (size_t)k * stride;
        v = x[o] - fcp[o] * v;
        x[o] = v;
    }
}

// Two-ended factored solve: the same systems eliminated from both ends at
// once ("twisted" factorization), two lanes per system, so each lane's
// dependent chain is half as long.  Rows k < h = N/2 keep the forward
// factors (a_k, 1/pivot_k) and c'_k of the one-ended solve; rows k >= h are
// eliminated upward from the last row: pivot'_k = b_k - c_k a'_{k+1},
// a'_k = a_k / pivot'_k, stored as (c_k, 1/pivot'_k) and a'_k.  The two
// half-sweeps meet in a 2 x 2 system for x_{h-1}, x_h.
__device__ __forceinline__ void lu2_factor_lane(int N, const float4 *eq, float2 *fai, float *fcp, size_t stride) {
    const int h = N / 2;
    float cp = 0.f;
    for (int k = 0; k < h; ++k) {
        const float4 e = eq[k];
        const float inv = frcp(e.y - e.x * cp);
        cp = e.z * inv;
        fai[k * stride] = make_float2(e.x, inv);
        fcp[k * stride] = cp;
    }
    float ap = 0.f;
    for (int k = N - 1; k >= h; --k) {
        const float4 e = eq[k];
        const float inv = frcp(e.y - e.z * ap);
        ap = e.x * inv;
        fai[k * stride] = make_float2(e.z, inv);
        fcp[k * stride] = ap;
    }
}

// acc <- (r_k - f.x acc) f.y over `count` unknowns from k0 in direction dir,
// each result stored to x_k; loads in blocks as in lu_solve_lane.
__device__ __forceinline__ float lu2_sweep(int k0, int dir, int count, const float *r, const float2 *fai, float *x,
                                           size_t stride) {
    float acc = 0.f;
    int i = 0;
    for (; i + LU_U <= count; i += LU_U) {
        float rr[LU_U];
        float2 ai[LU_U];
#pragma unroll
        for (int u = 0; u < LU_U; ++u) {
            const size_t o = (size_t)(k0 + dir * (i + u)) * stride;
            rr[u] = r[o];
            ai[u] = fai[o];
        }
#pragma unroll
        for (int u = 0; u < LU_U; ++u) {
            acc = (rr[u] - ai[u].x * acc) * ai[u].y;
            x[(size_t)(k0 + dir * (i + u)) * stride] = acc;
        }
    }
    for (; i < count; ++i) {
        const size_t o = (size_t)(k0 + dir * i) * stride;
        const float2 ai = fai[o];
        acc = (r[o] - ai.x * acc) * ai.y;
        x[o] = acc;
    }
    return acc;
}

// v <- x_k - c_k v over `count` unknowns from k0 in direction dir.
__device__ __forceinline__ void lu2_back(float v, int k0, int dir, int count, const float *fcp, float *x,
                                         size_t stride) {
    int i = 0;
    for (; i + LU_U <= count; i += LU_U) {
        float xx[LU_U], cc[LU_U];
#pragma unroll
        for (int u = 0; u < LU_U; ++u) {
            const size_t o = (size_t)(k0 + dir * (i + u)) * stride;
            xx[u] = x[o];
            cc[u] = fcp[o];
        }
#pragma unroll
        for (int u = 0; u < LU_U; ++u) {
            v = xx[u] - cc[u] * v;
            x[(size_t)(k0 + dir * (i + u)) * stride] = v;
        }
    }
    for (; i < count; ++i) {
        const size_t o = (size_t)(k0 + dir * i) * stride;
        v = x[o] - fcp[o] * v;
        x[o] = v;
    }
}

// One lane of a lane pair (top: rows 0 .. h-1, bottom: rows h .. N-1).
__device__ __forceinline__ void lu2_solve_lane(int N, bool top, const float *r, const float2 *fai,
                                               const float *fcp, float *x, size_t stride) {
    const int h = N / 2;
    const float acc = top ? lu2_sweep(0, 1, h, r, fai, x, stride) : lu2_sweep(N - 1, -1, N - h, r, fai, x, stride);
    const float cm = fcp[(size_t)(top ? h - 1 : h) * stride];  // c'_{h-1} (top) or a'_h (bottom)
    const float acc_o = __shfl_xor(acc, 1), cm_o = __shfl_xor(cm, 1);
    const float dp = top ? acc : acc_o, cp = top ? cm : cm_o;   // x_{h-1} + cp x_h = dp
    const float eq = top ? acc_o : acc, ap = top ? cm_o : cm;   // x_h + ap x_{h-1} = eq
    const float xl = (dp - cp * eq) * frcp(1.f - cp * ap);      // x_{h-1}
    const float xh = eq - ap * xl;                              // x_h
    if (top) {
        x[(size_t)(h - 1) * stride] = xl;
        lu2_back(xl, h - 2, -1, h - 1, fcp, x, stride);
    } else {
        x[(size_t)h * stride] = xh;
        lu2_back(xh, h + 1, 1, N - h - 1, fcp, x, stride);
    }
}

// Waves 0 .. xw-1 take the row systems, the rest the column systems.
__device__ __forceinline__ void lu_factor_body_impl(const SolveArgs &A, float *lux, float *luy, int wave, int lane,
                                                    bool two_ended) {
    const Dom &d = A.d;
    const int xw = (d.ny + 63) / 64;
    if (wave < xw) {
        const int j = wave * 64 + lane;
        const size_t n = (size_t)d.nu * d.ny;
        if (j < d.ny) {
            float2 *fai = reinterpret_cast<float2 *>(lux) + j;
            if (two_ended) lu2_factor_lane(d.nu, A.redx + (size_t)j * d.nu, fai, lux + 2 * n + j, d.ny);
            else lu_factor_lane(d.nu, A.redx + (size_t)j * d.nu, fai, lux + 2 * n + j, d.ny);
        }
    } else {
        const int i = (wave - xw) * 64 + lane;
        const size_t n = (size_t)d.nv * d.nx;
        if (i < d.nx) {
            float2 *fai = reinterpret_cast<float2 *>(luy) + i;
            if (two_ended) lu2_factor_lane(d.nv, A.redy + (size_t)i * d.nv, fai, luy + 2 * n + i, d.nx);
            else lu_factor_lane(d.nv, A.redy + (size_t)i * d.nv, fai, luy + 2 * n + i, d.nx);
        }
    }
}
__device__ __forceinline__ void lu_factor_body(const SolveArgs &A, float *lux, float *luy, int wave, int lane) {
    lu_factor_body_impl(A, lux, luy, wave, lane, false);
}

// Unknowns of one system per wave in the workgroup form of the factored solve.
constexpr int LUR = 32;
constexpr int LUW_MAX = 16;  // waves per workgroup (1024 threads): systems up to LUR x LUW_MAX
constexpr int LUS = 64;      // systems per workgroup, one a lane (32, with lanes l and l + 32
                             // on the same system, doubles the workgroups and gains nothing)

// The workgroup form of the one-ended sweeps, for systems of at most
// LUR x (waves in the workgroup) unknowns: a workgroup takes 64 systems, lane
// l of every wave system s0 + l, and wave q unknowns q LUR .. q LUR + LUR - 1
// of all 64, so every load and store covers 64 consecutive systems of one
// row of the interleaved layout, and the whole system sits in registers
// after one round trip.  The chain then runs wave by wave, handing the
// running value on through LDS between workgroup barriers: forward from
// wave 0, back from the last.  Same operations in the same order as
// lu_solve_lane (same bits).  Lanes past the last system compute on a copy
// of it and store nothing, so every wave reaches every barrier.
// Raw buffer access: a resource (base, size in bytes) in SGPRs, a per-lane
// byte offset and a wave-uniform byte offset, so that no per-lane 64-bit
// address is formed or kept; every offset used below is in range.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t bres(const void *p, size_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float bld(__amdgpu_buffer_rsrc_t r, unsigned vo, int so) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
}
__device__ __forceinline__ float2 bld2(__amdgpu_buffer_rsrc_t r, unsigned vo, int so) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0);
    return make_float2(__uint_as_float(v[0]), __uint_as_float(v[1]));
}
__device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, unsigned vo, int so, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, vo, so, 0);
}

// Workgroup barrier that waits only for the wave's LDS operations: the
// waves hand each other nothing through global memory here, so loads and
// stores in flight may stay in flight across it (a full __syncthreads
// would wait for every one of them at every hand-off).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

__device__ __forceinline__ void luw_solve(int N, int nsys, int s0, const float *r, const float2 *fai, const float *fcp,
                                          float *x, float *slot) {
    const int lane = threadIdx.x & 63;
    const int q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int G = blockDim.x >> 6;
    const int s = min(s0 + lane % LUS, nsys - 1);
    const bool live = lane < LUS && s0 + lane < nsys;
    const int k0 = q * LUR;
    const size_t n = (size_t)N * nsys;
    const auto br = bres(r, 4 * n), bf = bres(fai, 8 * n), bc = bres(fcp, 4 * n), bx = bres(x, 4 * n);
    const unsigned o4 = 4u * (unsigned)s, o8 = 8u * (unsigned)s;
    auto row = [&](int u) { return min(k0 + u, N - 1) * nsys; };  // wave-uniform
    // Rows past the system's end get y = 0 and factors (a, 1/pivot) = (-1, 1),
    // c' = -1, which pass the running value on exactly; the last row gets
    // c' = 0 (its back step gives x_{N-1} itself).  So every wave runs its
    // part without conditions.
    float y[LUR], cc[LUR];
    float2 ai[LUR];
#pragma unroll
    for (int u = 0; u < LUR; ++u) {
        const float yv = bld(br, o4, 4 * row(u));
        const float2 av = bld2(bf, o8, 8 * row(u));
        const bool in = k0 + u < N;
        y[u] = in ? yv : 0.f;
        ai[u] = in ? av : make_float2(-1.f, 1.f);
    }
    // Only the chain itself runs while the other waves wait: the values are
    // complete before the wave starts waiting (the empty asm takes them as
    // operands), and the loads and stores that need not precede a hand-off
    // follow it.
#pragma unroll
    for (int u = 0; u < LUR; ++u) asm volatile("" ::"v"(y[u]), "v"(ai[u].x), "v"(ai[u].y));
    // Every wave passes G barriers per sweep; wave q does its part between
    // its q-th and (q+1)-th (forward) or after the (G-1-q)-th (back).
    for (int t = 0; t < q; ++t) lds_barrier();
    {
        float acc = q ? slot[lane] : 0.f;
#pragma unroll
        for (int u = 0; u < LUR; ++u) {
            acc = (y[u] - ai[u].x * acc) * ai[u].y;
            y[u] = acc;
        }
        slot[lane] = acc;
    }
    lds_barrier();
#pragma unroll
    for (int u = 0; u < LUR; ++u) {
        const float cv = bld(bc, o4, 4 * row(u));
        cc[u] = k0 + u < N - 1 ? cv : k0 + u == N - 1 ? 0.f : -1.f;
    }
    for (int t = q + 1; t < G; ++t) lds_barrier();
    // the slot now holds y_{N-1} = x_{N-1}
#pragma unroll
    for (int u = 0; u < LUR; ++u) asm volatile("" ::"v"(cc[u]));
    for (int t = G - 1; t > q; --t) lds_barrier();
    {
        float acc = slot[lane];
#pragma unroll
        for (int u = LUR - 1; u >= 0; --u) {
            acc = y[u] - cc[u] * acc;
            y[u] = acc;
        }
        slot[lane] = acc;
    }
    lds_barrier();
    if (live) {
#pragma unroll
        for (int u = 0; u < LUR; ++u)
            if (k0 + u < N) bst(bx, o4, 4 * row(u), y[u]);
    }
    for (int t = q - 1; t >= 0; --t) lds_barrier();
}

// Workgroups 0 .. ceil(ny/LUS)-1 take the row systems, the rest the columns.
__device__ __forceinline__ void luw_solve_body(const SolveArgs &A, int wg, float *slot) {
    const Dom &d = A.d;
    const int xw = (d.ny + LUS - 1) / LUS;
    if (wg < xw)
        luw_solve(d.nu, d.ny, wg * LUS, reinterpret_cast<const float *>(A.redx),
                  reinterpret_cast<const float2 *>(A.lux), A.lux + 2 * (size_t)d.nu * d.ny, A.solx, slot);
    else
        luw_solve(d.nv, d.nx, (wg - xw) * LUS, reinterpret_cast<const float *>(A.redy),
                  reinterpret_cast<const float2 *>(A.luy), A.luy + 2 * (size_t)d.nv * d.nx, A.soly, slot);
}

__device__ __forceinline__ void lu_solve_body(const SolveArgs &A, int wave, int lane) {
    const Dom &d = A.d;
    const int xw = (d.ny + 63) / 64;
    if (wave < xw) {
        const int j = wave * 64 + lane;
        const size_t n = (size_t)d.nu * d.ny;
        if (j < d.ny)
            lu_solve_lane(d.nu, reinterpret_cast<const float *>(A.redx) + j, reinterpret_cast<const float2 *>(A.lux) + j,
                          A.lux + 2 * n + j, A.solx + j, d.ny);
    } else {
        const int i = (wave - xw) * 64 + lane;
        const size_t n = (size_t)d.nv * d.nx;
        if (i < d.nx)
            lu_solve_lane(d.nv, reinterpret_cast<const float *>(A.redy) + i, reinterpret_cast<const float2 *>(A.luy) + i,
                          A.luy + 2 * n + i, A.soly + i, d.nx);
    }
}

// Lane pairs (2q: top half, 2q + 1: bottom half) per system; waves
// 0 .. xw-1 take the row systems, the rest the column systems.
__device__ __forceinline__ void lu2_solve_body(const SolveArgs &A, int wave, int lane) {
    const Dom &d = A.d;
    const int xw = (2 * d.ny + 63) / 64;
    if (wave < xw) {
        const int l = wave * 64 + lane, j = l >> 1;
        const size_t n = (size_t)d.nu * d.ny;
        if (j < d.ny)
            lu2_solve_lane(d.nu, (l & 1) == 0, reinterpret_cast<const float *>(A.redx) + j,
                           reinterpret_cast<const float2 *>(A.lux) + j, A.lux + 2 * n + j, A.solx + j, d.ny);
    } else {
        const int l = (wave - xw) * 64 + lane, i = l >> 1;
        const size_t n = (size_t)d.nv * d.nx;
        if (i < d.nx)
            lu2_solve_lane(d.nv, (l & 1) == 0, reinterpret_cast<const float *>(A.redy) + i,
                           reinterpret_cast<const float2 *>(A.luy) + i, A.luy + 2 * n + i, A.soly + i, d.nx);
    }
}


__global__ __launch_bounds__(64) void k_lu_factor(SolveArgs A, float *lux, float *luy) {
    lu_factor_body(A, lux, luy, blockIdx.x, threadIdx.x);
}
__global__ __launch_bounds__(64) void k_lu_solve(SolveArgs A) { lu_solve_body(A, blockIdx.x, threadIdx.x); }
__global__ __launch_bounds__(64 * LUW_MAX) void k_luw_solve(SolveArgs A) {
    __shared__ float slot[64];
    luw_solve_body(A, blockIdx.x, slot);
}
__global__ __launch_bounds__(64) void k_lu2_factor(SolveArgs A, float *lux, float *luy) {
    lu_factor_body_impl(A, lux, luy, blockIdx.x, threadIdx.x, true);
}
__global__ __launch_bounds__(64) void k_lu2_solve(SolveArgs A) { lu2_solve_body(A, blockIdx.x, threadIdx.x); }

// Parallel cyclic reduction of one reduced system (rows first, then
// columns): each thread keeps its equations (k = tid + j * PCR_NT) in
// registers; one LDS copy of the system (dynamic size N) is read, then
// overwritten, per reduction level.
// PNT threads per system (64, 128 or 256): a tuning choice between more
// equations held per thread and more threads per barrier; EPL (a power of
// two, PNT * EPL >= N) equations per thread at most, so the register array
// is sized for the actual systems.
constexpr int PCR_NT = 128;  // default
// One PCR level for equation e with its neighbours m (stride below) and p
// (stride above), identity rows standing in past the system's ends: both
// PCR forms call it, so they give the same bits.
__device__ __forceinline__ float4 pcr_combine(float4 e, float4 m, float4 p) {
    const float al = -e.x * frcp(m.y), ga = -e.z * frcp(p.y);
    return make_float4(al * m.x, e.y + al * m.z + ga * p.x, ga * p.z, e.w + al * m.w + ga * p.w);
}
// One reduced system of N equations (sub, diag, super, rhs) from src; solutions to dst.
template <int PNT, int PCR_EPL>
__device__ __forceinline__ void pcr_solve(int N, const float4 *src, float *dst, float4 *buf) {
    const int tid = threadIdx.x;
    const int nmine = (N - tid + PNT - 1) / PNT;
    float4 eq[PCR_EPL];
#pragma unroll
    for (int j = 0; j < PCR_EPL; ++j)
        if (j < nmine) {
            eq[j] = src[tid + j * PNT];
            buf[tid + j * PNT] = eq[j];
        }
    __syncthreads();
    const float4 id = make_float4(0.f, 1.f, 0.f, 0.f);
    for (int st = 1; st < N; st <<= 1) {
#pragma unroll
        for (int j = 0; j < PCR_EPL; ++j)
            if (j < nmine) {
                const int k = tid + j * PNT;
                const float4 e = eq[j];
                const float4 m = k - st >= 0 ? buf[k - st] : id;
                const float4 p = k + st < N ? buf[k + st] : id;
                eq[j] = pcr_combine(e, m, p);
            }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PCR_EPL; ++j)
            if (j < nmine) buf[tid + j * PNT] = eq[j];
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < PCR_EPL; ++j)
        if (j < nmine) dst[tid + j * PNT] = eq[j].w / eq[j].y;
}

// PCR of one reduced system on a single wave, with no LDS array and no
// barrier: equation k = lane + 64 j sits in register j of its lane.  At a
// level of stride st < 64 the neighbours k - st and k + st are in lane
// (lane -+ st) mod 64, register j or the next one out, and come by lane
// shuffles (ds_bpermute); at st >= 64 they are the lane's own registers
// j -+ st / 64.  The levels are unrolled, so every register index is a
// compile-time constant.  Systems of up to 64 EPL unknowns.
__device__ __forceinline__ float4 shfl4(float4 v, int src) {
    return make_float4(__shfl(v.x, src), __shfl(v.y, src), __shfl(v.z, src), __shfl(v.w, src));
}
// Component-wise choice between two equations (a select of values: a ?: on
// the vectors themselves can become a select of addresses, which puts the
// register arrays in scratch memory).
__device__ __forceinline__ float4 sel4(bool c, float4 a, float4 b) {
    return make_float4(c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z, c ? a.w : b.w);
}
// One level (stride 2^LV) of the wave form, for every equation of the lane.
// Below stride 64 every neighbour is fetched by shuffles before any equation
// changes, so the update runs in place; from 64 on the neighbours are the
// lane's own registers and the new equations go to a fresh array first.
template <int EPL, int LV>
__device__ __forceinline__ void pcrw_level(int N, int lane, float4 (&eq)[EPL]) {
    constexpr int st = 1 << LV;
    const float4 id = make_float4(0.f, 1.f, 0.f, 0.f);
    if constexpr (st < 64) {
        const int up = (lane + st) & 63, dn = (lane - st) & 63;
        float4 su[EPL], sd[EPL];  // equation j of lane up, of lane dn
#pragma unroll
        for (int j = 0; j < EPL; ++j) {
            su[j] = shfl4(eq[j], up);
            sd[j] = shfl4(eq[j], dn);
        }
#pragma unroll
        for (int j = 0; j < EPL; ++j) {
            const int k = lane + 64 * j;
            const float4 hi = sel4(lane + st < 64, su[j], j + 1 < EPL ? su[j + 1] : id);
            const float4 lo = sel4(lane >= st, sd[j], j > 0 ? sd[j - 1] : id);
            eq[j] = pcr_combine(eq[j], sel4(k - st >= 0, lo, id), sel4(k + st < N, hi, id));
        }
    } else {
        constexpr int q = st / 64;
        float4 nw[EPL];
#pragma unroll
        for (int j = 0; j < EPL; ++j) {
            const int k = lane + 64 * j;
            const float4 hi = j + q < EPL ? eq[j + q] : id, lo = j >= q ? eq[j - q] : id;
            nw[j] = pcr_combine(eq[j], sel4(k - st >= 0, lo, id), sel4(k + st < N, hi, id));
        }
#pragma unroll
        for (int j = 0; j < EPL; ++j) eq[j] = nw[j];
    }
}
template <int EPL, int LV>
__device__ __forceinline__ void pcrw_levels(int N, int lane, float4 (&eq)[EPL]) {
    if constexpr ((1 << LV) < 64 * EPL) {
        if ((1 << LV) < N) {
            pcrw_level<EPL, LV>(N, lane, eq);
            pcrw_levels<EPL, LV + 1>(N, lane, eq);
        }
    }
}
template <int EPL>
__device__ __forceinline__ void pcrw_solve(int N, const float4 *src, float *dst) {
    const int lane = threadIdx.x & 63;
    const float4 id = make_float4(0.f, 1.f, 0.f, 0.f);
    float4 eq[EPL];
#pragma unroll
    for (int j = 0; j < EPL; ++j) {
        const int k = lane + 64 * j;
        eq[j] = sel4(k < N, src[k < N ? k : 0], id);
    }
    pcrw_levels<EPL, 0>(N, lane, eq);
#pragma unroll
    for (int j = 0; j < EPL; ++j) {
        const int k = lane + 64 * j;
        if (k < N) dst[k] = eq[j].w / eq[j].y;
    }
}
constexpr int PCRW_EPL_MAX = 8;  // the wave form takes systems of up to 512 unknowns

template <int EPL>
__global__ __launch_bounds__(64) void k_pcrw(SolveArgs A) {
    const Dom &d = A.d;
    const int sys = blockIdx.x;
    if (sys < d.ny) pcrw_solve<EPL>(d.nu, A.redx + (size_t)sys * d.nu, A.solx + (size_t)sys * d.nu);
    else pcrw_solve<EPL>(d.nv, A.redy + (size_t)(sys - d.ny) * d.nv, A.soly + (size_t)(sys - d.ny) * d.nv);
}

// System sys: rows 0..ny-1 (x direction), then columns.
template <int PNT, int EPL>
__device__ __forceinline__ void pcr_body(const SolveArgs &A, float4 *buf, int sys) {
    const Dom &d = A.d;
    if (sys < d.ny) pcr_solve<PNT, EPL>(d.nu, A.redx + (size_t)sys * d.nu, A.solx + (size_t)sys * d.nu, buf);
    else pcr_solve<PNT, EPL>(d.nv, A.redy + (size_t)(sys - d.ny) * d.nv, A.soly + (size_t)(sys - d.ny) * d.nv, buf);
}

template <int PNT, int EPL>
__global__ __launch_bounds__(PNT) void k_pcr(SolveArgs A) {
    extern __shared__ float4 buf[];
    pcr_body<PNT, EPL>(A, buf, blockIdx.x);
}

template <int T = NT>
__device__ __forceinline__ void expand_body(const SolveArgs &A, SolveTile &s, int bx, int by) {
    constexpr int CPT = cells_per_thread<T>();
    const Dom &d = A.d;
    const int tid = threadIdx.x;
    const int i0 = bx * TX, j0 = by * TY;
    // epilogue inputs first: in flight while the tile is staged
    float pre_e[CPT], pre_p[CPT], pre_q[CPT];
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int k = tid + m * T, cx = k % TX, cy = k / TX, i = i0 + cx, j = j0 + cy;
        const int o = j * d.pitch + i;
        const bool in = i < d.nx && j < d.ny;
        pre_e[m] = in ? A.eta[o] : 0.f;
        pre_p[m] = in ? A.pbase[o] : 0.f;
        pre_q[m] = in ? A.qbase[o] : 0.f;
    }
    stage_tile<T>(A, s, i0, j0);
    if (A.nlsw) {
        // identity systems (eq. 21-22 with the dispersive coefficients zero):
        // the partitioned solve would return the increments unchanged
    } else if (tid < 64) {
        const int row = tid % 16, seg = tid / 16, k0 = seg * MX;
        const int k = 2 * (bx * (TX / MX) + seg), j = j0 + row;
        float x0 = 0.f, xl = 0.f;
        if (A.layout) {
            if (j < d.ny) {
                x0 = A.solx[(size_t)k * d.ny + j];
                xl = A.solx[(size_t)(k + 1) * d.ny + j];
            }
        } else {
            const float *sol = A.solx + (size_t)j * d.nu + k;
            x0 = sol[0];
            xl = sol[1];
        }
        float a[MX], b[MX], c[MX];
        float *r = &s.rx[row][k0];
        seg_coefs<MX>(A, s, i0, j0, 0, k0, row, a, b, c, r, 1);  // boundary rows fold into r, as in the reduction
        seg_expand<MX>(r, 1, a, b, c, x0, xl);
    } else if (tid < 128) {
        const int col = tid - 64;
        const int i = i0 + col;
        float x0 = 0.f, xl = 0.f;
        if (A.layout) {
            if (i < d.nx) {
                x0 = A.soly[(size_t)(2 * by) * d.nx + i];
                xl = A.soly[(size_t)(2 * by + 1) * d.nx + i];
            }
        } else {
            const float *sol = A.soly + (size_t)i * d.nv + 2 * by;
            x0 = sol[0];
            xl = sol[1];
        }
        float a[TY], b[TY], c[TY];
        float *r = &s.ry[0][col];
        seg_coefs<TY>(A, s, i0, j0, 1, col, 0, a, b, c, r, TXP);
        seg_expand<TY>(r, TXP, a, b, c, x0, xl);
    }
    __syncthreads();
    int bad = 0;
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int k = tid + m * T, cx = k % TX, cy = k / TX, i = i0 + cx, j = j0 + cy;
        if (i >= d.nx || j >= d.ny) continue;
        const int o = j * d.pitch + i;
        float P = pre_p[m] + s.rx[cy][cx], Q = pre_q[m] + s.ry[cy][cx], e = pre_e[m];
        // unclamped still-water depth of the cell (negative on land)
        const float Dc = 0.25f * ((s.cz[cy + 1][cx + 1] + s.cz[cy + 1][cx + 2]) +
                                  (s.cz[cy + 2][cx + 1] + s.cz[cy + 2][cx + 2]));
        const float h = e + Dc, h2 = h * h, h4 = h2 * h2;
        if (h4 < d.eps) {  // shoreline: discharge = h * desingularized velocity
            // h^4 + eps rounded once (an explicit fused multiply-add, so that
            // every kernel this body is compiled into rounds it alike)
            const float f = 1.41421356237f * h2 * frsq(fmaf(h2, h2, d.eps));
            P *= f;
            Q *= f;
        }
        if (A.sponge && Dc > 0.f) {
            float gm = 1.f;
            if (d.side[0].type == BC_SPONGE)
                gm *= sponge_factor(sponge_gamma((i + 0.5f) * d.dx, d.side[0].width * d.dx), d.side[0].expo);
            if (d.side[1].type == BC_SPONGE)
                gm *= sponge_factor(sponge_gamma((d.nx - i - 0.5f) * d.dx, d.side[1].width * d.dx), d.side[1].expo);
            if (d.side[2].type == BC_SPONGE)
                gm *= sponge_factor(sponge_gamma((j + 0.5f) * d.dy, d.side[2].width * d.dy), d.side[2].expo);
            if (d.side[3].type == BC_SPONGE)
                gm *= sponge_factor(sponge_gamma((d.ny - j - 0.5f) * d.dy, d.side[3].width * d.dy), d.side[3].expo);
            if (gm != 1.f) {
                e *= gm;
                P *= gm;
                Q *= gm;
                A.eta[o] = e;
            }
        }
        bad |= !(isfinite(P) && isfinite(Q) && isfinite(e));
        A.pout[o] = P;
        A.qout[o] = Q;
    }
    // one atomic per wave: a non-finite state must not serialize every thread
    // of the launch on the health word
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(A.health, 1);
}

__global__ __launch_bounds__(NT) void k_expand(SolveArgs A) {
    __shared__ SolveTile s;
    expand_body(A, s, blockIdx.x, blockIdx.y);
}

}  // namespace ws
