// ws_kernels.hpp -- the gfx950 kernels of one predictor/corrector pass.
//
// A pass is four launches:
//   k_stencil  one workgroup per 64x16 tile: halo-staged (LDS) state, KP07
//              face fluxes, dispersive and friction terms, time integration;
//              writes the new surface and the increments U* - U*^n,
//              V* - V*^n (the solves work in delta form: T (P - P^n) =
//              U* - U*^n, algebraically the same system, whose right-hand
//              side is O(dt F) instead of O(P), so single precision loses
//              far less in the solve).
//   k_reduce   per tile: coefficients of eq. 23 from the bathymetry, and the
//              elimination of every 64-cell row segment and 16-cell column
//              segment down to its first and last unknowns (partition
//              method); writes the eliminated interior values in place and
//              two reduced equations per segment.
//   k_pcr      one workgroup per row and per column system: parallel cyclic
//              reduction of the reduced tridiagonal system in LDS.
//   k_expand   per tile: back substitution of every segment from its solved
//              end values, P = P^n + dP, Q = Q^n + dQ, shoreline fix (and the
//              sponge after the last pass).
#pragma once
#include "ws_device.hpp"

namespace ws {

constexpr int HX = TX + 4, HY = TY + 4;  // state halo tile (2 ghost cells per side)
constexpr int CX = TX + 5, CY = TY + 5;  // corner tile of the halo

struct StencilArgs {
    Dom d;
    const float *ein, *pin, *qin;      // estimate (the state itself for the predictor)
    float *eout, *rx, *ry;             // new surface, U* - U*^n, V* - V*^n
    float *hE, *hF, *hG, *hFs, *hGs;   // history level n (predictors write it)
    const float *E1, *F1, *G1, *Fs1, *Gs1;  // level n-1
    const float *E2, *F2, *G2, *Fs2, *Gs2;  // level n-2
    float *Se, *SU, *SV;               // corrector bases (eta, U* and V* increments)
    double t;                          // time of the ghost values
    float dt, x0, x1, x2;              // step, F* extrapolation weights
    int kind;                          // 0 Euler predictor, 1 AB3 predictor, 2 AM4 corrector
    int write_S;
};

__device__ __forceinline__ float dcell4(float a, float b, float c, float d) {
    return fmaxf(0.25f * ((a + b) + (c + d)), 0.f);
}

__global__ __launch_bounds__(NT) void k_stencil(StencilArgs A) {
    __shared__ float se[HY][HX], sp[HY][HX], sq[HY][HX];
    __shared__ float sD[CY][CX];
    __shared__ float fx[3][TY][TX + 1];
    __shared__ float fy[3][TY + 1][TX];
    const Dom &d = A.d;
    const int tid = threadIdx.x;
    const int i0 = blockIdx.x * TX, j0 = blockIdx.y * TY;
    const float th = d.theta, g = d.g, eps = d.eps;

    for (int k = tid; k < HX * HY; k += NT) {
        int lx = k % HX, ly = k / HX;
        float e, p, q;
        load_cell(d, A.ein, A.pin, A.qin, i0 + lx - 2, j0 + ly - 2, A.t, e, p, q);
        se[ly][lx] = e;
        sp[ly][lx] = p;
        sq[ly][lx] = q;
    }
    for (int k = tid; k < CX * CY; k += NT) {
        int lx = k % CX, ly = k / CX;
        sD[ly][lx] = corner_D(d, i0 + lx - 2, j0 + ly - 2);
    }
    __syncthreads();

    // x-faces: face fi lies between local cells fi+1 and fi+2 of row fj+2
    for (int k = tid; k < (TX + 1) * TY; k += NT) {
        int fi = k % (TX + 1), fj = k / (TX + 1);
        int ly = fj + 2, a = fi + 1, b = fi + 2;
        float Dwa = 0.5f * (sD[ly][a] + sD[ly + 1][a]);
        float Df = 0.5f * (sD[ly][b] + sD[ly + 1][b]);
        float Deb = 0.5f * (sD[ly][b + 1] + sD[ly + 1][b + 1]);
        F3 lo, hiL, loR, hi;
        reconstruct(se[ly][a - 1], se[ly][a], se[ly][a + 1], sp[ly][a - 1], sp[ly][a], sp[ly][a + 1],
                    sq[ly][a - 1], sq[ly][a], sq[ly][a + 1], Dwa, Df, th, lo, hiL);
        reconstruct(se[ly][b - 1], se[ly][b], se[ly][b + 1], sp[ly][b - 1], sp[ly][b], sp[ly][b + 1],
                    sq[ly][b - 1], sq[ly][b], sq[ly][b + 1], Df, Deb, th, loR, hi);
        float H0, H1, H2;
        cu_flux(g, eps, Df, hiL, loR, H0, H1, H2);
        fx[0][fj][fi] = H0;
        fx[1][fj][fi] = H1;
        fx[2][fj][fi] = H2;
    }
    // y-faces: face fj lies between local rows fj+1 and fj+2 of column fi+2;
    // the normal discharge is Q
    for (int k = tid; k < TX * (TY + 1); k += NT) {
        int fi = k % TX, fj = k / TX;
        int lx = fi + 2, a = fj + 1, b = fj + 2;
        float Dsa = 0.5f * (sD[a][lx] + sD[a][lx + 1]);
        float Df = 0.5f * (sD[b][lx] + sD[b][lx + 1]);
        float Dnb = 0.5f * (sD[b + 1][lx] + sD[b + 1][lx + 1]);
        F3 lo, hiL, loR, hi;
        reconstruct(se[a - 1][lx], se[a][lx], se[a + 1][lx], sq[a - 1][lx], sq[a][lx], sq[a + 1][lx],
                    sp[a - 1][lx], sp[a][lx], sp[a + 1][lx], Dsa, Df, th, lo, hiL);
        reconstruct(se[b - 1][lx], se[b][lx], se[b + 1][lx], sq[b - 1][lx], sq[b][lx], sq[b + 1][lx],
                    sp[b - 1][lx], sp[b][lx], sp[b + 1][lx], Df, Dnb, th, loR, hi);
        float H0, H1, H2;
        cu_flux(g, eps, Df, hiL, loR, H0, H1, H2);
        fy[0][fj][fi] = H0;
        fy[1][fj][fi] = H2;  // x-momentum (tangential)
        fy[2][fj][fi] = H1;  // y-momentum (normal)
    }
    __syncthreads();

    const float rdx = d.rdx, rdy = d.rdy, Bd = d.Bd, B3 = d.Bd + 1.f / 3.f;
    const int cx = tid % TX;
    for (int cy = tid / TX; cy < TY; cy += NT / TX) {
        const int i = i0 + cx, j = j0 + cy;
        if (i >= d.nx || j >= d.ny) continue;
        const int lx = cx + 2, ly = cy + 2;
        const float c00 = sD[ly][lx], c10 = sD[ly][lx + 1], c01 = sD[ly + 1][lx], c11 = sD[ly + 1][lx + 1];
        const float Dc = 0.25f * ((c00 + c10) + (c01 + c11));
        const float Dw = 0.5f * (c00 + c01), De = 0.5f * (c10 + c11);
        const float Ds = 0.5f * (c00 + c10), Dn = 0.5f * (c01 + c11);
        const float e0 = se[ly][lx], p0 = sp[ly][lx], q0 = sq[ly][lx];

        float E = -(fx[0][cy][cx + 1] - fx[0][cy][cx]) * rdx - (fy[0][cy + 1][cx] - fy[0][cy][cx]) * rdy;
        float F = -(fx[1][cy][cx + 1] - fx[1][cy][cx]) * rdx - (fy[1][cy + 1][cx] - fy[1][cy][cx]) * rdy +
                  g * (De - Dw) * rdx * e0;
        float G = -(fx[2][cy][cx + 1] - fx[2][cy][cx]) * rdx - (fy[2][cy + 1][cx] - fy[2][cy][cx]) * rdy +
                  g * (Dn - Ds) * rdy * e0;
        float Fs = 0.f, Gs = 0.f;

        const float dep = fmaxf(Dc, 0.f);
        const float dxm = dcell4(sD[ly][lx - 1], sD[ly][lx], sD[ly + 1][lx - 1], sD[ly + 1][lx]);
        const float dxp = dcell4(sD[ly][lx + 1], sD[ly][lx + 2], sD[ly + 1][lx + 1], sD[ly + 1][lx + 2]);
        const float dym = dcell4(sD[ly - 1][lx], sD[ly - 1][lx + 1], sD[ly][lx], sD[ly][lx + 1]);
        const float dyp = dcell4(sD[ly + 1][lx], sD[ly + 1][lx + 1], sD[ly + 2][lx], sD[ly + 2][lx + 1]);
        const float ddx = (dxp - dxm) * 0.5f * rdx, ddy = (dyp - dym) * 0.5f * rdy;

        if (d.model == BSNQ) {
            const float em1 = se[ly][lx - 1], ep1 = se[ly][lx + 1], em2 = se[ly][lx - 2], ep2 = se[ly][lx + 2];
            const float fm1 = se[ly - 1][lx], fp1 = se[ly + 1][lx], fm2 = se[ly - 2][lx], fp2 = se[ly + 2][lx];
            const float epp = se[ly + 1][lx + 1], epm = se[ly - 1][lx + 1];
            const float emp = se[ly + 1][lx - 1], emm = se[ly - 1][lx - 1];
            const float exx = (ep1 - 2.f * e0 + em1) * rdx * rdx;
            const float eyy = (fp1 - 2.f * e0 + fm1) * rdy * rdy;
            const float exy = (epp - epm - emp + emm) * 0.25f * rdx * rdy;
            const float exxx = (ep2 - 2.f * ep1 + 2.f * em1 - em2) * 0.5f * rdx * rdx * rdx;
            const float eyyy = (fp2 - 2.f * fp1 + 2.f * fm1 - fm2) * 0.5f * rdy * rdy * rdy;
            const float exyy = ((epp - 2.f * ep1 + epm) - (emp - 2.f * em1 + emm)) * 0.5f * rdx * rdy * rdy;
            const float exxy = ((epp - 2.f * fp1 + emp) - (epm - 2.f * fm1 + emm)) * 0.5f * rdx * rdx * rdy;
            const float gb = Bd * g * dep * dep;
            F += gb * (dep * (exxx + exyy) + ddx * (2.f * exx + eyy) + ddy * exy);
            G += gb * (dep * (eyyy + exxy) + ddy * (2.f * eyy + exx) + ddx * exy);
            const float Px = (sp[ly][lx + 1] - sp[ly][lx - 1]) * 0.5f * rdx;
            const float Py = (sp[ly + 1][lx] - sp[ly - 1][lx]) * 0.5f * rdy;
            const float Pxy = (sp[ly + 1][lx + 1] - sp[ly - 1][lx + 1] - sp[ly + 1][lx - 1] + sp[ly - 1][lx - 1]) *
                              0.25f * rdx * rdy;
            const float Qx = (sq[ly][lx + 1] - sq[ly][lx - 1]) * 0.5f * rdx;
            const float Qy = (sq[ly + 1][lx] - sq[ly - 1][lx]) * 0.5f * rdy;
            const float Qxy = (sq[ly + 1][lx + 1] - sq[ly - 1][lx + 1] - sq[ly + 1][lx - 1] + sq[ly - 1][lx - 1]) *
                              0.25f * rdx * rdy;
            Fs = dep * (ddx * Qy + ddy * Qx) * (1.f / 6.f) + B3 * dep * dep * Qxy;
            Gs = dep * (ddy * Px + ddx * Py) * (1.f / 6.f) + B3 * dep * dep * Pxy;
        }
        if (d.friction != FRIC_NONE) {
            const float h = fmaxf(e0 + Dc, 0.f), h2 = h * h, h4 = h2 * h2;
            const float inv_h = 1.41421356237f * h * rsqrtf(h4 + fmaxf(h4, eps));
            float fc = d.fcoef;
            if (d.friction == FRIC_MANNING) fc = g * d.fcoef * d.fcoef * cbrtf(inv_h);
            const float k = fc * sqrtf(p0 * p0 + q0 * q0) * inv_h * inv_h;
            F -= k * p0;
            G -= k * q0;
        }

        const size_t o = (size_t)j * d.pitch + i;
        float en, U = 0.f, V = 0.f;   // increments of U*, V* over the step
        if (A.kind != 2) {
            A.hE[o] = E;
            A.hF[o] = F;
            A.hG[o] = G;
            A.hFs[o] = Fs;
            A.hGs[o] = Gs;
        }
        const float dt = A.dt;
        if (A.kind == 0) {
            en = e0 + dt * E;
            U += dt * F;
            V += dt * G;
        } else if (A.kind == 1) {
            const float e1 = A.E1[o], e2 = A.E2[o], f1 = A.F1[o], f2 = A.F2[o], g1 = A.G1[o], g2 = A.G2[o];
            const float fs1 = A.Fs1[o], gs1 = A.Gs1[o];
            const float fs2 = A.x2 != 0.f ? A.Fs2[o] : 0.f, gs2 = A.x2 != 0.f ? A.Gs2[o] : 0.f;
            const float c12 = dt * (1.f / 12.f), c24 = dt * (1.f / 24.f);
            if (A.write_S) {
                A.Se[o] = e0 + c24 * (19.f * E - 5.f * e1 + e2);
                A.SU[o] = U + c24 * (19.f * F - 5.f * f1 + f2) - Fs;
                A.SV[o] = V + c24 * (19.f * G - 5.f * g1 + g2) - Gs;
            }
            en = e0 + c12 * (23.f * E - 16.f * e1 + 5.f * e2);
            U = U + c12 * (23.f * F - 16.f * f1 + 5.f * f2) + (A.x0 * Fs + A.x1 * fs1 + A.x2 * fs2);
            V = V + c12 * (23.f * G - 16.f * g1 + 5.f * g2) + (A.x0 * Gs + A.x1 * gs1 + A.x2 * gs2);
        } else {
            const float c9 = dt * (9.f / 24.f);
            en = A.Se[o] + c9 * E;
            U = A.SU[o] + c9 * F + Fs;
            V = A.SV[o] + c9 * G + Gs;
        }
        A.eout[o] = fmaxf(en, -Dc);
        A.rx[o] = U;
        A.ry[o] = V;
    }
}

// ------------------------------------------------------------- solver parts
struct SolveArgs {
    Dom d;
    float *rx, *ry;            // right-hand sides in, eliminated segment interiors out
    float4 *redx, *redy;       // reduced equations (sub, diag, super, rhs) per unknown
    float *solx, *soly;        // reduced solutions
    float *eta, *pout, *qout;  // new surface (read; sponge writes it), new P, Q
    const float *pbase, *qbase;  // P^n, Q^n of the step
    int *health;
    double t0, t1;             // wave-maker ghosts of the boundary rows: t^n and t^{n+1}
    int sponge;
};

struct SolveTile {
    float rx[TY][TX], ry[TY][TX];
    float D[TY + 3][TX + 3];   // corners of cells -1..TX, -1..TY
    float xa[TY][TX], xb[TY][TX], xc[TY][TX];
    float ya[TY][TX], yb[TY][TX], yc[TY][TX];
};

__device__ __forceinline__ float tile_dcell(const SolveTile &s, int cx, int cy) {
    return dcell4(s.D[cy + 1][cx + 1], s.D[cy + 1][cx + 2], s.D[cy + 2][cx + 1], s.D[cy + 2][cx + 2]);
}

// Load the tile's corners and fill the row (x) and column (y) coefficients of
// eq. 23 for every cell, folding the boundary rows: behind a wall the ghost
// is the odd mirror of the first unknown (diagonal -= off-diagonal), behind a
// wave maker it is the maker's discharge, known, so its change over the step
// moves to the right-hand side of the delta-form system (when adjust_rhs).
// Padding cells become identity rows with zero right-hand side.
// Change of a wave maker's ghost discharge (P if comp == 0, else Q) from t^n
// to t^{n+1} at (x, y).
__device__ inline float ghost_change(const SideDev &sd, double x, double y, const SolveArgs &A, int comp) {
    float e0, p0, q0, e1, p1, q1;
    wave_eval(sd, x, y, A.t0, e0, p0, q0);
    wave_eval(sd, x, y, A.t1, e1, p1, q1);
    return comp == 0 ? p1 - p0 : q1 - q0;
}

__device__ void fill_coefs(const SolveArgs &A, SolveTile &s, int i0, int j0, bool adjust_rhs) {
    const Dom &d = A.d;
    const int tid = threadIdx.x;
    for (int k = tid; k < (TX + 3) * (TY + 3); k += NT) {
        int lx = k % (TX + 3), ly = k / (TX + 3);
        s.D[ly][lx] = corner_D(d, i0 + lx - 1, j0 + ly - 1);
    }
    __syncthreads();
    for (int k = tid; k < TX * TY; k += NT) {
        const int cx = k % TX, cy = k / TX, i = i0 + cx, j = j0 + cy;
        float a = 0.f, b = 1.f, c = 0.f, a2 = 0.f, b2 = 1.f, c2 = 0.f;
        if (i < d.nx && j < d.ny) {
            const float dep = tile_dcell(s, cx, cy);
            const float ddx = (tile_dcell(s, cx + 1, cy) - tile_dcell(s, cx - 1, cy)) * 0.5f * d.rdx;
            const float ddy = (tile_dcell(s, cx, cy + 1) - tile_dcell(s, cx, cy - 1)) * 0.5f * d.rdy;
            tri_coef(d, dep, ddx, d.rdx, a, b, c);
            tri_coef(d, dep, ddy, d.rdy, a2, b2, c2);
            if (i == 0) {
                if (is_wall(d, 0)) b -= a;
                else if (adjust_rhs)
                    s.rx[cy][cx] -= a * ghost_change(d.side[0], -0.5 * d.dx, (j + 0.5) * (double)d.dy, A, 0);
                a = 0.f;
            }
            if (i == d.nx - 1) {
                if (is_wall(d, 1)) b -= c;
                else if (adjust_rhs)
                    s.rx[cy][cx] -= c * ghost_change(d.side[1], (d.nx + 0.5) * (double)d.dx, (j + 0.5) * (double)d.dy, A, 0);
                c = 0.f;
            }
            if (j == 0) {
                if (is_wall(d, 2)) b2 -= a2;
                else if (adjust_rhs)
                    s.ry[cy][cx] -= a2 * ghost_change(d.side[2], (i + 0.5) * (double)d.dx, -0.5 * d.dy, A, 1);
                a2 = 0.f;
            }
            if (j == d.ny - 1) {
                if (is_wall(d, 3)) b2 -= c2;
                else if (adjust_rhs)
                    s.ry[cy][cx] -= c2 * ghost_change(d.side[3], (i + 0.5) * (double)d.dx, (d.ny + 0.5) * (double)d.dy, A, 1);
                c2 = 0.f;
            }
        } else if (adjust_rhs) {
            s.rx[cy][cx] = 0.f;
            s.ry[cy][cx] = 0.f;
        }
        s.xa[cy][cx] = a;
        s.xb[cy][cx] = b;
        s.xc[cy][cx] = c;
        s.ya[cy][cx] = a2;
        s.yb[cy][cx] = b2;
        s.yc[cy][cx] = c2;
    }
    __syncthreads();
}

// Partition-method elimination of one segment of M unknowns (stride st in
// LDS): afterwards every interior row k reads  a_k x_0 + b_k x_k + c_k x_{M-1}
// = r_k (r overwritten), and the first and last rows are returned as reduced
// equations coupling (x_{-1}, x_0, x_{M-1}) and (x_0, x_{M-1}, x_M).
template <int M>
__device__ void seg_eliminate(float *r, float *a, float *b, const float *c, int st, float4 &first,
                              float4 &last) {
    for (int k = 2; k <= M - 2; ++k) {  // forward: eliminate x_{k-1} in favour of x_0
        const float f = a[k * st] / b[(k - 1) * st];
        a[k * st] = -f * a[(k - 1) * st];
        b[k * st] = b[k * st] - f * c[(k - 1) * st];
        r[k * st] = r[k * st] - f * r[(k - 1) * st];
    }
    {
        const float f = a[(M - 1) * st] / b[(M - 2) * st];
        last = make_float4(-f * a[(M - 2) * st], b[(M - 1) * st] - f * c[(M - 2) * st],
                           c[(M - 1) * st], r[(M - 1) * st] - f * r[(M - 2) * st]);
    }
    float ah = a[(M - 2) * st], bh = b[(M - 2) * st], ch = c[(M - 2) * st], rh = r[(M - 2) * st];
    for (int k = M - 3; k >= 1; --k) {  // backward: eliminate x_{k+1} in favour of x_{M-1}
        const float f = c[k * st] / bh;
        ah = a[k * st] - f * ah;
        bh = b[k * st];
        ch = -f * ch;
        rh = r[k * st] - f * rh;
        r[k * st] = rh;
    }
    const float f = c[0] / bh;
    first = make_float4(a[0], b[0] - f * ah, -f * ch, r[0] - f * rh);
}

// Back substitution of one segment from its solved end values x0, xl; r holds
// the eliminated interior values on entry and the solution on exit.
template <int M>
__device__ void seg_expand(float *r, float *a, float *b, const float *c, int st, float x0, float xl) {
    for (int k = 2; k <= M - 2; ++k) {
        const float f = a[k * st] / b[(k - 1) * st];
        a[k * st] = -f * a[(k - 1) * st];
        b[k * st] = b[k * st] - f * c[(k - 1) * st];
    }
    float ah = a[(M - 2) * st], bh = b[(M - 2) * st], ch = c[(M - 2) * st];
    r[(M - 2) * st] = (r[(M - 2) * st] - ah * x0 - ch * xl) / bh;
    for (int k = M - 3; k >= 1; --k) {
        const float f = c[k * st] / bh;
        ah = a[k * st] - f * ah;
        bh = b[k * st];
        ch = -f * ch;
        r[k * st] = (r[k * st] - ah * x0 - ch * xl) / bh;
    }
    r[0] = x0;
    r[(M - 1) * st] = xl;
}

__global__ __launch_bounds__(NT) void k_reduce(SolveArgs A) {
    __shared__ SolveTile s;
    const Dom &d = A.d;
    const int tid = threadIdx.x, bx = blockIdx.x, by = blockIdx.y;
    const int i0 = bx * TX, j0 = by * TY;
    for (int k = tid; k < TX * TY; k += NT) {
        const int cx = k % TX, cy = k / TX;
        const size_t o = (size_t)(j0 + cy) * d.pitch + i0 + cx;
        s.rx[cy][cx] = A.rx[o];
        s.ry[cy][cx] = A.ry[o];
    }
    fill_coefs(A, s, i0, j0, true);
    if (tid < TY) {
        float4 first, last;
        seg_eliminate<TX>(&s.rx[tid][0], &s.xa[tid][0], &s.xb[tid][0], &s.xc[tid][0], 1, first, last);
        float4 *red = A.redx + (size_t)(j0 + tid) * d.nu + 2 * bx;
        red[0] = first;
        red[1] = last;
    } else if (tid >= 64 && tid < 64 + TX) {
        const int c = tid - 64;
        float4 first, last;
        seg_eliminate<TY>(&s.ry[0][c], &s.ya[0][c], &s.yb[0][c], &s.yc[0][c], TX, first, last);
        float4 *red = A.redy + (size_t)(i0 + c) * d.nv + 2 * by;
        red[0] = first;
        red[1] = last;
    }
    __syncthreads();
    for (int k = tid; k < TX * TY; k += NT) {
        const int cx = k % TX, cy = k / TX;
        const size_t o = (size_t)(j0 + cy) * d.pitch + i0 + cx;
        A.rx[o] = s.rx[cy][cx];
        A.ry[o] = s.ry[cy][cx];
    }
}

// Parallel cyclic reduction of one reduced system (rows first, then columns).
__global__ __launch_bounds__(NT) void k_pcr(SolveArgs A) {
    __shared__ float4 buf[2][NRED_MAX];
    const Dom &d = A.d;
    int sys = blockIdx.x, N;
    const float4 *src;
    float *dst;
    if (sys < d.ny) {
        N = d.nu;
        src = A.redx + (size_t)sys * N;
        dst = A.solx + (size_t)sys * N;
    } else {
        sys -= d.ny;
        N = d.nv;
        src = A.redy + (size_t)sys * N;
        dst = A.soly + (size_t)sys * N;
    }
    const int tid = threadIdx.x;
    for (int k = tid; k < N; k += NT) buf[0][k] = src[k];
    __syncthreads();
    int cur = 0;
    const float4 id = make_float4(0.f, 1.f, 0.f, 0.f);
    for (int st = 1; st < N; st <<= 1) {
        for (int k = tid; k < N; k += NT) {
            const float4 e = buf[cur][k];
            const float4 m = k - st >= 0 ? buf[cur][k - st] : id;
            const float4 p = k + st < N ? buf[cur][k + st] : id;
            const float al = -e.x / m.y, ga = -e.z / p.y;
            buf[cur ^ 1][k] = make_float4(al * m.x, e.y + al * m.z + ga * p.x, ga * p.z,
                                          e.w + al * m.w + ga * p.w);
        }
        cur ^= 1;
        __syncthreads();
    }
    for (int k = tid; k < N; k += NT) dst[k] = buf[cur][k].w / buf[cur][k].y;
}

__global__ __launch_bounds__(NT) void k_expand(SolveArgs A) {
    __shared__ SolveTile s;
    const Dom &d = A.d;
    const int tid = threadIdx.x, bx = blockIdx.x, by = blockIdx.y;
    const int i0 = bx * TX, j0 = by * TY;
    for (int k = tid; k < TX * TY; k += NT) {
        const int cx = k % TX, cy = k / TX;
        const size_t o = (size_t)(j0 + cy) * d.pitch + i0 + cx;
        s.rx[cy][cx] = A.rx[o];
        s.ry[cy][cx] = A.ry[o];
    }
    fill_coefs(A, s, i0, j0, false);
    if (tid < TY) {
        const float *sol = A.solx + (size_t)(j0 + tid) * d.nu + 2 * bx;
        seg_expand<TX>(&s.rx[tid][0], &s.xa[tid][0], &s.xb[tid][0], &s.xc[tid][0], 1, sol[0], sol[1]);
    } else if (tid >= 64 && tid < 64 + TX) {
        const int c = tid - 64;
        const float *sol = A.soly + (size_t)(i0 + c) * d.nv + 2 * by;
        seg_expand<TY>(&s.ry[0][c], &s.ya[0][c], &s.yb[0][c], &s.yc[0][c], TX, sol[0], sol[1]);
    }
    __syncthreads();
    int bad = 0;
    for (int k = tid; k < TX * TY; k += NT) {
        const int cx = k % TX, cy = k / TX, i = i0 + cx, j = j0 + cy;
        if (i >= d.nx || j >= d.ny) continue;
        const size_t o = (size_t)j * d.pitch + i;
        float P = A.pbase[o] + s.rx[cy][cx], Q = A.qbase[o] + s.ry[cy][cx], e = A.eta[o];
        const float Dc = 0.25f * ((s.D[cy + 1][cx + 1] + s.D[cy + 1][cx + 2]) +
                                  (s.D[cy + 2][cx + 1] + s.D[cy + 2][cx + 2]));
        const float h = e + Dc, h2 = h * h, h4 = h2 * h2;
        if (h4 < d.eps) {  // shoreline: discharge = h * desingularized velocity
            const float f = 1.41421356237f * h2 * rsqrtf(h4 + d.eps);
            P *= f;
            Q *= f;
        }
        if (A.sponge && Dc > 0.f) {
            float gm = 1.f;
            if (d.side[0].type == BC_SPONGE) gm *= sponge_gamma((i + 0.5f) * d.dx, d.side[0].width * d.dx);
            if (d.side[1].type == BC_SPONGE) gm *= sponge_gamma((d.nx - i - 0.5f) * d.dx, d.side[1].width * d.dx);
            if (d.side[2].type == BC_SPONGE) gm *= sponge_gamma((j + 0.5f) * d.dy, d.side[2].width * d.dy);
            if (d.side[3].type == BC_SPONGE) gm *= sponge_gamma((d.ny - j - 0.5f) * d.dy, d.side[3].width * d.dy);
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
    if (bad) atomicOr(A.health, 1);
}

}  // namespace ws
