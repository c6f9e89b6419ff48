/*
 * wave_oracle.c -- FP64 CPU oracle for one time step of the hybrid
 * finite-volume / finite-difference extended-Boussinesq solver described by
 * Tavakkol & Lynett, "Celeris: A GPU-accelerated open source software with a
 * Boussinesq-type wave solver ..." (arXiv:1611.05984).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the parity reference for the GPU
 * library and the CPU baseline of the benchmark.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg load it.  It shares no
 * source, header, table or helper with the GPU path.
 *
 * Plain and slow on purpose: every quantity is evaluated where it is used, the
 * step runs in the order the paper describes it, arithmetic is IEEE double
 * with no contraction (built with -ffp-contract=off, no fast-math).  OpenMP
 * only splits the outer row/column loops; results do not depend on it.
 *
 * Grid (the paper's uniform Cartesian cells, sec. 2.2): cell (i,j), i in
 * [0,nx), j in [0,ny), centre ((i+1/2)dx, (j+1/2)dy).  Two ghost layers on
 * every side (sec. 2.4).  Bathymetry z is sampled at cell corners (i dx, j dy)
 * and is continuous and bilinear, as the central-upwind scheme (KP07) it
 * follows assumes; the paper does not say how its bathymetry texture is
 * sampled, so this corner sampling is a reading of the paper, not its
 * statement.
 *
 * Parity pins live in tests/ (lake at rest, volume, solitary wave, linear
 * dispersion relation, dam breaks, symmetries, polynomial exactness,
 * tridiagonal solver vs a library solver).  The constants theta (minmod),
 * the flux guard and the start-up/wet-dry/sponge/wave-maker details the paper
 * leaves open are "parity unpinned" against the paper: both sides implement
 * the same stated reading.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXC 256 /* wave components per side */

enum { OR_BSNQ = 0, OR_NLSW = 1 };
enum { OR_FRIC_NONE = 0, OR_FRIC_QUAD = 1, OR_FRIC_MANNING = 2 };
enum { OR_WEST = 0, OR_EAST = 1, OR_SOUTH = 2, OR_NORTH = 3 };
enum { OR_SOLID = 0, OR_SPONGE = 1, OR_WAVES = 2 };
enum { OR_EDIT_WATER = 0, OR_EDIT_TERRAIN = 1 };

typedef struct {
    int32_t nx, ny;
    int32_t n_corr;   /* corrector iterations after the predictor (Fig. 2 sample: 2) */
    int32_t model;    /* OR_BSNQ or OR_NLSW (sec. 3.2)                               */
    int32_t friction; /* none / quadratic eq. (31) / Manning eq. (32)                */
    int32_t fstar_extrap; /* predictor extrapolation of F*, G*: 2 = quadratic as
                             printed in eqs. (16)-(17), 1 = linear (default), 0 = none */
    double dx, dy, dt;
    double g;         /* gravitational acceleration                                  */
    double ws;        /* still water surface elevation w_s (sec. 2.1)                */
    double Bdisp;     /* dispersion calibration coefficient B = 1/15 (sec. 2.1)      */
    double theta;     /* generalized minmod parameter (sec. 2.2 step 1)              */
    double eps;       /* desingularization tolerance epsilon of eq. (14)             */
    double fcoef;     /* friction coefficient f (eq. 31) or Manning n (eq. 32)       */
} or_params;

typedef struct {
    int type, width, ncomp;
    double expo; /* sponge: exponent s of the damping factor gamma^s (1 = eq. 30) */
    double reflect; /* sponge: target reflection coefficient it was set with (0 = eq. 30) */
    double amp[OR_MAXC], omega[OR_MAXC], k[OR_MAXC], c[OR_MAXC];
    double dirx[OR_MAXC], diry[OR_MAXC], phase[OR_MAXC];
} or_side;

typedef struct {
    or_params p;
    or_side side[4];
    int sx;            /* row stride of ghosted cell arrays: nx + 4 */
    int zx;            /* row stride of the ghosted corner array: nx + 5 */
    double *z;         /* corner bathymetry, corners -2..nx+2 x -2..ny+2 */
    double *w, *P, *Q; /* state, ghosted cell arrays */
    double *E[3], *F[3], *G[3], *Fs[3], *Gs[3]; /* right-hand-side history ring */
    int64_t step;      /* number of completed time steps since the last start */
    double t;
    int health;        /* 0 ok, 1 non-finite state seen */
    /* corrector iteration until convergence (sec. 2.3): off while tol_w <= 0 */
    double tol_w, tol_pq;     /* largest allowed change of w, of P and Q       */
    int last_corr;            /* correctors the last step ran                  */
    int64_t total_corr;       /* correctors run since the tolerance was set    */
    double last_dw, last_dpq; /* changes measured after the last corrector     */
} or_domain;

/* ---------------------------------------------------------------- indexing */
static size_t CI(const or_domain *D, int i, int j) {
    return (size_t)(j + 2) * (size_t)D->sx + (size_t)(i + 2);
}
static size_t ZI(const or_domain *D, int ci, int cj) {
    return (size_t)(cj + 2) * (size_t)D->zx + (size_t)(ci + 2);
}
static size_t ncells_ghosted(const or_domain *D) {
    return (size_t)(D->p.nx + 4) * (size_t)(D->p.ny + 4);
}

/* ------------------------------------------------------------- bathymetry */
/* Continuous bilinear bottom from corner values: the bottom at a face is the
 * mean of the face's two corners, the cell value is the mean of its four
 * corners (the mean of its two x-faces and of its two y-faces). */
static double zc(const or_domain *D, int ci, int cj) { return D->z[ZI(D, ci, cj)]; }
static double bface_x(const or_domain *D, int i, int j) { /* west face of cell (i,j) */
    return 0.5 * (zc(D, i, j) + zc(D, i, j + 1));
}
static double bface_y(const or_domain *D, int i, int j) { /* south face of cell (i,j) */
    return 0.5 * (zc(D, i, j) + zc(D, i + 1, j));
}
static double bcell(const or_domain *D, int i, int j) {
    return 0.25 * (zc(D, i, j) + zc(D, i + 1, j) + zc(D, i, j + 1) + zc(D, i + 1, j + 1));
}
/* Still water depth d (sec. 2.1): w_s - z where that is positive, 0 on land
 * (so the equations reduce to NLSW there). */
static double dstill(const or_domain *D, int i, int j) {
    double d = D->p.ws - bcell(D, i, j);
    return d > 0.0 ? d : 0.0;
}

static int is_wall(int type) { return type == OR_SOLID || type == OR_SPONGE; }

/* Ghost corners: mirrored (even) across solid and sponge sides, copied
 * (constant) across wave-maker sides.  x-sides first, then y-sides over all
 * corner columns. */
static void fill_bathy_ghosts(or_domain *D) {
    int nx = D->p.nx, ny = D->p.ny;
    for (int cj = 0; cj <= ny; ++cj)
        for (int g = 1; g <= 2; ++g) {
            D->z[ZI(D, -g, cj)] = is_wall(D->side[OR_WEST].type) ? zc(D, g, cj) : zc(D, 0, cj);
            D->z[ZI(D, nx + g, cj)] =
                is_wall(D->side[OR_EAST].type) ? zc(D, nx - g, cj) : zc(D, nx, cj);
        }
    for (int ci = -2; ci <= nx + 2; ++ci)
        for (int g = 1; g <= 2; ++g) {
            D->z[ZI(D, ci, -g)] = is_wall(D->side[OR_SOUTH].type) ? zc(D, ci, g) : zc(D, ci, 0);
            D->z[ZI(D, ci, ny + g)] =
                is_wall(D->side[OR_NORTH].type) ? zc(D, ci, ny - g) : zc(D, ci, ny);
        }
}

/* ------------------------------------------------------- boundary forcing */
/* Wave-maker values at a point, sec. 2.4.2: each component m contributes
 * eta_m = a sin(omega t - k_x x - k_y y + phi), P_m = c cos(theta) eta_m,
 * Q_m = c sin(theta) eta_m (eqs. 25-28); components superpose linearly. */
static void wave_values(const or_side *s, double ws, double x, double y, double t, double *w,
                        double *P, double *Q) {
    double eta = 0.0, p = 0.0, q = 0.0;
    for (int m = 0; m < s->ncomp; ++m) {
        double e = s->amp[m] *
                   sin(s->omega[m] * t - s->k[m] * (s->dirx[m] * x + s->diry[m] * y) + s->phase[m]);
        eta += e;
        p += s->c[m] * s->dirx[m] * e;
        q += s->c[m] * s->diry[m] * e;
    }
    *w = ws + eta;
    *P = p;
    *Q = q;
}

/* Eckart's approximate dispersion relation, eq. (29). */
double or_eckart_k(double omega, double d, double g) {
    double x = omega * omega * d / g;
    return (omega * omega / g) * sqrt(1.0 / tanh(x));
}

/* Two ghost layers per side (sec. 2.4).  Solid walls and sponge edges mirror
 * the two nearest interior cells about the boundary face (sec. 2.4.1): w and
 * the tangential discharge are even, the normal discharge is odd, so
 * (P,Q).n = 0 and grad(w).n = 0 (eq. 24).  Wave-maker sides assign the
 * analytic values of sec. 2.4.2 at the ghost cell centres.  A ghost is a
 * function of its position: it is first reflected across every wall side it
 * lies behind (flipping the sign of that side's normal discharge); if it then
 * still lies behind a wave-maker side, the maker's values at the reflected
 * position are used (an x-side maker if it lies behind two makers). */
static void ghost_value(const or_domain *D, const double *w, const double *P, const double *Q,
                        int i, int j, double t, double *gw, double *gp, double *gq) {
    const int nx = D->p.nx, ny = D->p.ny;
    double sp = 1.0, sq = 1.0;
    if (i < 0 && is_wall(D->side[OR_WEST].type)) { i = -1 - i; sp = -sp; }
    if (i >= nx && is_wall(D->side[OR_EAST].type)) { i = 2 * nx - 1 - i; sp = -sp; }
    if (j < 0 && is_wall(D->side[OR_SOUTH].type)) { j = -1 - j; sq = -sq; }
    if (j >= ny && is_wall(D->side[OR_NORTH].type)) { j = 2 * ny - 1 - j; sq = -sq; }
    double vw, vp, vq;
    if (i >= 0 && i < nx && j >= 0 && j < ny) {
        size_t c = CI(D, i, j);
        vw = w[c]; vp = P[c]; vq = Q[c];
    } else {
        int side = i < 0 ? OR_WEST : i >= nx ? OR_EAST : j < 0 ? OR_SOUTH : OR_NORTH;
        wave_values(&D->side[side], D->p.ws, (i + 0.5) * D->p.dx, (j + 0.5) * D->p.dy, t, &vw,
                    &vp, &vq);
    }
    *gw = vw;
    *gp = sp * vp;
    *gq = sq * vq;
}

static void fill_ghosts(or_domain *D, double *w, double *P, double *Q, double t) {
    const int nx = D->p.nx, ny = D->p.ny;
    for (int j = -2; j < ny + 2; ++j)
        for (int i = -2; i < nx + 2; ++i) {
            if (i >= 0 && i < nx && j >= 0 && j < ny) continue;
            size_t c = CI(D, i, j);
            ghost_value(D, w, P, Q, i, j, t, &w[c], &P[c], &Q[c]);
        }
}

/* --------------------------------------------- KP07 reconstruction, sec 2.2 */
/* Generalized minmod of three arguments. */
double or_minmod3(double a, double b, double c) {
    if (a > 0.0 && b > 0.0 && c > 0.0) return fmin(a, fmin(b, c));
    if (a < 0.0 && b < 0.0 && c < 0.0) return fmax(a, fmax(b, c));
    return 0.0;
}
/* Limited undivided slope of the middle value (step 1: generalized minmod on
 * the one-sided and central differences, theta in [1,2]). */
static double limited_slope(double um, double u0, double up, double theta) {
    return or_minmod3(theta * (u0 - um), 0.5 * (up - um), theta * (up - u0));
}

typedef struct { double w, n, t; } face_state; /* surface, normal and tangential discharge */

/* Step 1 + step 2 (first half): linear reconstruction of (w, n, t) at the two
 * faces of a cell along one direction, then the conservative positivity
 * correction of w against the face bottoms: if the reconstruction puts w
 * below the bottom at one face, that face is set to the bottom and the other
 * face takes the value that keeps the cell mean. */
static void reconstruct(double wm, double w0, double wp, double nm, double n0, double np, double tm,
                        double t0, double tp, double b_lo, double b_hi, double theta,
                        face_state *lo, face_state *hi) {
    double sw = limited_slope(wm, w0, wp, theta);
    double sn = limited_slope(nm, n0, np, theta);
    double st = limited_slope(tm, t0, tp, theta);
    lo->w = w0 - 0.5 * sw;
    hi->w = w0 + 0.5 * sw;
    lo->n = n0 - 0.5 * sn;
    hi->n = n0 + 0.5 * sn;
    lo->t = t0 - 0.5 * st;
    hi->t = t0 + 0.5 * st;
    if (hi->w < b_hi) {
        hi->w = b_hi;
        lo->w = 2.0 * w0 - b_hi;
    } else if (lo->w < b_lo) {
        lo->w = b_lo;
        hi->w = 2.0 * w0 - b_lo;
    }
}

/* Eq. (14): desingularized velocity u = sqrt(2) h m / sqrt(h^4 + max(h^4, eps)). */
double or_desing(double h, double m, double eps) {
    double h4 = h * h * h * h;
    return M_SQRT2 * h * m / sqrt(h4 + fmax(h4, eps));
}

/* Step 3: central-upwind numerical flux (KP07) at one face, written for the
 * face-normal direction: returns (mass, normal momentum, tangential momentum)
 * fluxes.  The physical flux is (h u, h u^2 + g h^2/2, h u v) with u the
 * normal and v the tangential velocity (the F and G of eq. 1); the discharges
 * are recomputed as h*u, h*v after desingularization; the numerical
 * diffusion acts on (w, h u, h v).  Where the one-sided local speeds
 * a+ - a- vanish (both sides dry) the flux is zero (guard 1e-10 m/s, the
 * paper gives none). */
void or_cu_flux(double g, double eps, double bf, const double L[3], const double R[3],
                double H[3]) {
    double hL = fmax(L[0] - bf, 0.0), hR = fmax(R[0] - bf, 0.0);
    double uL = or_desing(hL, L[1], eps), vL = or_desing(hL, L[2], eps);
    double uR = or_desing(hR, R[1], eps), vR = or_desing(hR, R[2], eps);
    double nL = hL * uL, tL = hL * vL, nR = hR * uR, tR = hR * vR;
    double cL = sqrt(g * hL), cR = sqrt(g * hR);
    double ap = fmax(fmax(uL + cL, uR + cR), 0.0);
    double am = fmin(fmin(uL - cL, uR - cR), 0.0);
    if (ap - am <= 1e-10) {
        H[0] = H[1] = H[2] = 0.0;
        return;
    }
    double FL[3] = {nL, nL * uL + 0.5 * g * hL * hL, nL * vL};
    double FR[3] = {nR, nR * uR + 0.5 * g * hR * hR, nR * vR};
    double UL[3] = {L[0], nL, tL};
    double UR[3] = {R[0], nR, tR};
    for (int k = 0; k < 3; ++k)
        H[k] = (ap * FL[k] - am * FR[k]) / (ap - am) + ap * am / (ap - am) * (UR[k] - UL[k]);
}

/* ----------------------------------------------- right-hand side, eqs 9-13 */
/* E, F, G of eqs. (9)-(11) and F*, G* of eqs. (12)-(13) for every interior
 * cell from a ghosted state whose ghosts are already filled.  Advective terms
 * and the bottom slope: KP07 fluxes + its well-balanced source (step 4),
 * S = -g (B_{i+1/2} - B_{i-1/2}) / dx * (w - B_i).  Dispersive terms (BSNQ
 * model only): second-order central differences added as sources (end of
 * sec. 2.2).  Friction: eq. (31)/(32) with 1/h^2 desingularized as in (14). */
static void rhs(const or_domain *D, const double *w, const double *P, const double *Q, double *E,
                double *F, double *G, double *Fs, double *Gs) {
    const int nx = D->p.nx, ny = D->p.ny;
    const double dx = D->p.dx, dy = D->p.dy, g = D->p.g, eps = D->p.eps, th = D->p.theta;
    double *Hx = malloc(sizeof(double) * 3 * (size_t)(nx + 1) * (size_t)ny);
    double *Hy = malloc(sizeof(double) * 3 * (size_t)nx * (size_t)(ny + 1));

    /* x-faces: face i is the west face of cell i, between cells i-1 and i */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i <= nx; ++i) {
            face_state lo, hiL, loR, hi;
            int a = i - 1, b = i;
            reconstruct(w[CI(D, a - 1, j)], w[CI(D, a, j)], w[CI(D, a + 1, j)], P[CI(D, a - 1, j)],
                        P[CI(D, a, j)], P[CI(D, a + 1, j)], Q[CI(D, a - 1, j)], Q[CI(D, a, j)],
                        Q[CI(D, a + 1, j)], bface_x(D, a, j), bface_x(D, a + 1, j), th, &lo, &hiL);
            reconstruct(w[CI(D, b - 1, j)], w[CI(D, b, j)], w[CI(D, b + 1, j)], P[CI(D, b - 1, j)],
                        P[CI(D, b, j)], P[CI(D, b + 1, j)], Q[CI(D, b - 1, j)], Q[CI(D, b, j)],
                        Q[CI(D, b + 1, j)], bface_x(D, b, j), bface_x(D, b + 1, j), th, &loR, &hi);
            double L[3] = {hiL.w, hiL.n, hiL.t}, R[3] = {loR.w, loR.n, loR.t};
            double *H = &Hx[3 * ((size_t)j * (nx + 1) + i)];
            or_cu_flux(g, eps, bface_x(D, i, j), L, R, H); /* (mass, x-mom, y-mom) */
        }
    /* y-faces: face j is the south face of cell j, between cells j-1 and j;
     * normal discharge is Q, tangential is P */
#pragma omp parallel for schedule(static)
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i < nx; ++i) {
            face_state lo, hiL, loR, hi;
            int a = j - 1, b = j;
            reconstruct(w[CI(D, i, a - 1)], w[CI(D, i, a)], w[CI(D, i, a + 1)], Q[CI(D, i, a - 1)],
                        Q[CI(D, i, a)], Q[CI(D, i, a + 1)], P[CI(D, i, a - 1)], P[CI(D, i, a)],
                        P[CI(D, i, a + 1)], bface_y(D, i, a), bface_y(D, i, a + 1), th, &lo, &hiL);
            reconstruct(w[CI(D, i, b - 1)], w[CI(D, i, b)], w[CI(D, i, b + 1)], Q[CI(D, i, b - 1)],
                        Q[CI(D, i, b)], Q[CI(D, i, b + 1)], P[CI(D, i, b - 1)], P[CI(D, i, b)],
                        P[CI(D, i, b + 1)], bface_y(D, i, b), bface_y(D, i, b + 1), th, &loR, &hi);
            double L[3] = {hiL.w, hiL.n, hiL.t}, R[3] = {loR.w, loR.n, loR.t};
            double *H = &Hy[3 * ((size_t)j * nx + i)];
            or_cu_flux(g, eps, bface_y(D, i, j), L, R, H); /* (mass, y-mom, x-mom) */
        }

    const double B = D->p.Bdisp, B3 = D->p.Bdisp + 1.0 / 3.0, ws = D->p.ws;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t c = CI(D, i, j);
            const double *Hw = &Hx[3 * ((size_t)j * (nx + 1) + i)];
            const double *He = &Hx[3 * ((size_t)j * (nx + 1) + i + 1)];
            const double *Hs = &Hy[3 * ((size_t)j * nx + i)];
            const double *Hn = &Hy[3 * ((size_t)(j + 1) * nx + i)];
            double depth_above_cell = w[c] - bcell(D, i, j);
            double e = -(He[0] - Hw[0]) / dx - (Hn[0] - Hs[0]) / dy;
            double f = -(He[1] - Hw[1]) / dx - (Hn[2] - Hs[2]) / dy -
                       g * (bface_x(D, i + 1, j) - bface_x(D, i, j)) / dx * depth_above_cell;
            double gg = -(He[2] - Hw[2]) / dx - (Hn[1] - Hs[1]) / dy -
                        g * (bface_y(D, i, j + 1) - bface_y(D, i, j)) / dy * depth_above_cell;
            double fs = 0.0, gs = 0.0;
            if (D->p.model == OR_BSNQ) {
                double d = dstill(D, i, j);
                double d_x = (dstill(D, i + 1, j) - dstill(D, i - 1, j)) / (2.0 * dx);
                double d_y = (dstill(D, i, j + 1) - dstill(D, i, j - 1)) / (2.0 * dy);
#define ETA(a, b) (w[CI(D, i + (a), j + (b))] - ws)
                double exx = (ETA(1, 0) - 2.0 * ETA(0, 0) + ETA(-1, 0)) / (dx * dx);
                double eyy = (ETA(0, 1) - 2.0 * ETA(0, 0) + ETA(0, -1)) / (dy * dy);
                double exy = (ETA(1, 1) - ETA(1, -1) - ETA(-1, 1) + ETA(-1, -1)) / (4.0 * dx * dy);
                double exxx =
                    (ETA(2, 0) - 2.0 * ETA(1, 0) + 2.0 * ETA(-1, 0) - ETA(-2, 0)) / (2.0 * dx * dx * dx);
                double eyyy =
                    (ETA(0, 2) - 2.0 * ETA(0, 1) + 2.0 * ETA(0, -1) - ETA(0, -2)) / (2.0 * dy * dy * dy);
                double exyy = ((ETA(1, 1) - 2.0 * ETA(1, 0) + ETA(1, -1)) -
                               (ETA(-1, 1) - 2.0 * ETA(-1, 0) + ETA(-1, -1))) /
                              (2.0 * dx * dy * dy);
                double exxy = ((ETA(1, 1) - 2.0 * ETA(0, 1) + ETA(-1, 1)) -
                               (ETA(1, -1) - 2.0 * ETA(0, -1) + ETA(-1, -1))) /
                              (2.0 * dx * dx * dy);
#undef ETA
                /* dispersive parts of eqs. (10) and (11) */
                f += B * g * d * d * d * (exxx + exyy) + B * g * d * d * (d_x * (2.0 * exx + eyy) + d_y * exy);
                gg += B * g * d * d * d * (eyyy + exxy) + B * g * d * d * (d_y * (2.0 * eyy + exx) + d_x * exy);
#define FLD(A, a, b) (A[CI(D, i + (a), j + (b))])
                double Px = (FLD(P, 1, 0) - FLD(P, -1, 0)) / (2.0 * dx);
                double Py = (FLD(P, 0, 1) - FLD(P, 0, -1)) / (2.0 * dy);
                double Pxy = (FLD(P, 1, 1) - FLD(P, 1, -1) - FLD(P, -1, 1) + FLD(P, -1, -1)) / (4.0 * dx * dy);
                double Qx = (FLD(Q, 1, 0) - FLD(Q, -1, 0)) / (2.0 * dx);
                double Qy = (FLD(Q, 0, 1) - FLD(Q, 0, -1)) / (2.0 * dy);
                double Qxy = (FLD(Q, 1, 1) - FLD(Q, 1, -1) - FLD(Q, -1, 1) + FLD(Q, -1, -1)) / (4.0 * dx * dy);
#undef FLD
                /* eq. (12) and eq. (13) (whose argument is P) */
                fs = d * d_x * Qy / 6.0 + d * d_y * Qx / 6.0 + B3 * d * d * Qxy;
                gs = d * d_y * Px / 6.0 + d * d_x * Py / 6.0 + B3 * d * d * Pxy;
            }
            if (D->p.friction != OR_FRIC_NONE) {
                double h = fmax(depth_above_cell, 0.0), h4 = h * h * h * h;
                double inv_h = M_SQRT2 * h / sqrt(h4 + fmax(h4, eps)); /* 1/h as in eq. (14) */
                double fc = D->p.fcoef;
                if (D->p.friction == OR_FRIC_MANNING) fc = g * D->p.fcoef * D->p.fcoef * cbrt(inv_h);
                double speed = sqrt(P[c] * P[c] + Q[c] * Q[c]);
                f -= fc * P[c] * speed * inv_h * inv_h;
                gg -= fc * Q[c] * speed * inv_h * inv_h;
            }
            E[c] = e;
            F[c] = f;
            G[c] = gg;
            Fs[c] = fs;
            Gs[c] = gs;
        }
    free(Hx);
    free(Hy);
}

/* --------------------------------------------- tridiagonal systems, eq. 23 */
/* Coefficients of eqs. (21)-(23) for one cell along one direction: spacing
 * h, still water depth d and its derivative dd along that direction. */
static void tri_coefs(const or_domain *D, double d, double dd, double h, double *A, double *Bm,
                      double *C) {
    if (D->p.model == OR_NLSW) {
        *A = 0.0;
        *Bm = 1.0;
        *C = 0.0;
        return;
    }
    double b3 = D->p.Bdisp + 1.0 / 3.0;
    *A = d * dd / (6.0 * h) - b3 * d * d / (h * h);
    *Bm = 1.0 + 2.0 * b3 * d * d / (h * h);
    *C = -d * dd / (6.0 * h) - b3 * d * d / (h * h);
}
static void row_coefs(const or_domain *D, int i, int j, double *A, double *Bm, double *C) {
    double d = dstill(D, i, j);
    double dd = (dstill(D, i + 1, j) - dstill(D, i - 1, j)) / (2.0 * D->p.dx);
    tri_coefs(D, d, dd, D->p.dx, A, Bm, C);
}
static void col_coefs(const or_domain *D, int i, int j, double *A, double *Bm, double *C) {
    double d = dstill(D, i, j);
    double dd = (dstill(D, i, j + 1) - dstill(D, i, j - 1)) / (2.0 * D->p.dy);
    tri_coefs(D, d, dd, D->p.dy, A, Bm, C);
}

/* Thomas algorithm (forward elimination, back substitution; sec. 3.3). */
void or_thomas(int n, const double *a, const double *b, const double *c, const double *r,
               double *x) {
    double *cp = malloc(sizeof(double) * (size_t)n), *dp = malloc(sizeof(double) * (size_t)n);
    cp[0] = c[0] / b[0];
    dp[0] = r[0] / b[0];
    for (int i = 1; i < n; ++i) {
        double m = b[i] - a[i] * cp[i - 1];
        cp[i] = c[i] / m;
        dp[i] = (r[i] - a[i] * dp[i - 1]) / m;
    }
    x[n - 1] = dp[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
    free(cp);
    free(dp);
}

/* U* = A P_{i-1} + B P_i + C P_{i+1} (eqs. 7 and 21 read as an operator on P),
 * V* likewise along y on Q, from a ghosted P, Q with filled ghosts. */
static void ustar(const or_domain *D, const double *P, const double *Q, double *U, double *V) {
    const int nx = D->p.nx, ny = D->p.ny;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double A, Bm, C;
            row_coefs(D, i, j, &A, &Bm, &C);
            U[CI(D, i, j)] = A * P[CI(D, i - 1, j)] + Bm * P[CI(D, i, j)] + C * P[CI(D, i + 1, j)];
            col_coefs(D, i, j, &A, &Bm, &C);
            V[CI(D, i, j)] = A * Q[CI(D, i, j - 1)] + Bm * Q[CI(D, i, j)] + C * Q[CI(D, i, j + 1)];
        }
}

/* Solve eq. (21) on every row for P and eq. (22) on every column for Q.  The
 * first and last unknowns couple to ghost values: behind a solid or sponge
 * side the ghost is the odd mirror (P_{-1} = -P_0), folded into the diagonal;
 * behind a wave-maker side it is the analytic value at time t, moved to the
 * right-hand side. */
static void solve_rows(const or_domain *D, const double *U, double *P, double t) {
    const int nx = D->p.nx, ny = D->p.ny;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
        double *a = malloc(sizeof(double) * 5 * (size_t)nx);
        double *b = a + nx, *c = b + nx, *r = c + nx, *x = r + nx;
        for (int i = 0; i < nx; ++i) {
            row_coefs(D, i, j, &a[i], &b[i], &c[i]);
            r[i] = U[CI(D, i, j)];
        }
        double gw, gp, gq;
        if (D->side[OR_WEST].type == OR_WAVES) {
            wave_values(&D->side[OR_WEST], D->p.ws, -0.5 * D->p.dx, (j + 0.5) * D->p.dy, t, &gw, &gp, &gq);
            r[0] -= a[0] * gp;
        } else {
            b[0] -= a[0];
        }
        a[0] = 0.0;
        if (D->side[OR_EAST].type == OR_WAVES) {
            wave_values(&D->side[OR_EAST], D->p.ws, (nx + 0.5) * D->p.dx, (j + 0.5) * D->p.dy, t, &gw, &gp, &gq);
            r[nx - 1] -= c[nx - 1] * gp;
        } else {
            b[nx - 1] -= c[nx - 1];
        }
        c[nx - 1] = 0.0;
        or_thomas(nx, a, b, c, r, x);
        for (int i = 0; i < nx; ++i) P[CI(D, i, j)] = x[i];
        free(a);
    }
}
static void solve_cols(const or_domain *D, const double *V, double *Q, double t) {
    const int nx = D->p.nx, ny = D->p.ny;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nx; ++i) {
        double *a = malloc(sizeof(double) * 5 * (size_t)ny);
        double *b = a + ny, *c = b + ny, *r = c + ny, *x = r + ny;
        for (int j = 0; j < ny; ++j) {
            col_coefs(D, i, j, &a[j], &b[j], &c[j]);
            r[j] = V[CI(D, i, j)];
        }
        double gw, gp, gq;
        if (D->side[OR_SOUTH].type == OR_WAVES) {
            wave_values(&D->side[OR_SOUTH], D->p.ws, (i + 0.5) * D->p.dx, -0.5 * D->p.dy, t, &gw, &gp, &gq);
            r[0] -= a[0] * gq;
        } else {
            b[0] -= a[0];
        }
        a[0] = 0.0;
        if (D->side[OR_NORTH].type == OR_WAVES) {
            wave_values(&D->side[OR_NORTH], D->p.ws, (i + 0.5) * D->p.dx, (ny + 0.5) * D->p.dy, t, &gw, &gp, &gq);
            r[ny - 1] -= c[ny - 1] * gq;
        } else {
            b[ny - 1] -= c[ny - 1];
        }
        c[ny - 1] = 0.0;
        or_thomas(ny, a, b, c, r, x);
        for (int j = 0; j < ny; ++j) Q[CI(D, i, j)] = x[j];
        free(a);
    }
}

/* ------------------------------------------------- wet/dry and sponge layer */
/* Moving shoreline.  The cell mean surface never goes below the cell bottom
 * (KP07 positivity needs w >= B; the multistep integrator does not guarantee
 * it, so it is clamped), and where the depth is below the desingularization
 * scale the discharges are recomputed as h*u with u from eq. (14) (KP07),
 * which leaves them unchanged wherever h^4 >= eps. */
static void dry_fix_w(const or_domain *D, double *w) {
#pragma omp parallel for schedule(static)
    for (int j = 0; j < D->p.ny; ++j)
        for (int i = 0; i < D->p.nx; ++i) {
            double b = bcell(D, i, j);
            if (w[CI(D, i, j)] < b) w[CI(D, i, j)] = b;
        }
}
static void dry_fix_pq(const or_domain *D, const double *w, double *P, double *Q) {
#pragma omp parallel for schedule(static)
    for (int j = 0; j < D->p.ny; ++j)
        for (int i = 0; i < D->p.nx; ++i) {
            size_t c = CI(D, i, j);
            double h = w[c] - bcell(D, i, j), h4 = h * h * h * h;
            if (h4 < D->p.eps) {
                double s = M_SQRT2 * h * h / sqrt(h4 + D->p.eps);
                P[c] *= s;
                Q[c] *= s;
            }
        }
}

/* Sponge layer damping coefficient, eq. (30), for a cell centre at normal
 * distance D from the absorbing boundary of a layer of width Ls. */
double or_sponge_gamma(double dist, double Ls) {
    if (dist >= Ls) return 1.0;
    return 0.5 * (1.0 + cos(M_PI * (Ls - dist) / Ls));
}
/* Damping factor of a sponge cell: gamma^s, s = 1 being eq. (30) itself and
 * s = 0 no damping (see or_set_sponge_reflect). */
static double sponge_factor(const or_side *s, double gamma) {
    return s->expo == 1.0 ? gamma : s->expo == 0.0 ? 1.0 : pow(gamma, s->expo);
}
static void sponge(const or_domain *D, double *w, double *P, double *Q) {
    const int nx = D->p.nx, ny = D->p.ny;
    const double dx = D->p.dx, dy = D->p.dy;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            if (dstill(D, i, j) <= 0.0) continue;
            double gm = 1.0;
            if (D->side[OR_WEST].type == OR_SPONGE)
                gm *= sponge_factor(&D->side[OR_WEST], or_sponge_gamma((i + 0.5) * dx, D->side[OR_WEST].width * dx));
            if (D->side[OR_EAST].type == OR_SPONGE)
                gm *= sponge_factor(&D->side[OR_EAST], or_sponge_gamma((nx - i - 0.5) * dx, D->side[OR_EAST].width * dx));
            if (D->side[OR_SOUTH].type == OR_SPONGE)
                gm *= sponge_factor(&D->side[OR_SOUTH], or_sponge_gamma((j + 0.5) * dy, D->side[OR_SOUTH].width * dy));
            if (D->side[OR_NORTH].type == OR_SPONGE)
                gm *= sponge_factor(&D->side[OR_NORTH], or_sponge_gamma((ny - j - 0.5) * dy, D->side[OR_NORTH].width * dy));
            if (gm == 1.0) continue;
            size_t c = CI(D, i, j);
            w[c] = D->p.ws + gm * (w[c] - D->p.ws);
            P[c] *= gm;
            Q[c] *= gm;
        }
}

/* ------------------------------------------------------------ time step */
static void check_health(or_domain *D) {
    for (int j = 0; j < D->p.ny; ++j)
        for (int i = 0; i < D->p.nx; ++i) {
            size_t c = CI(D, i, j);
            if (!isfinite(D->w[c]) || !isfinite(D->P[c]) || !isfinite(D->Q[c])) D->health = 1;
        }
}

/* One full time step t^n -> t^{n+1} (sec. 2.3).
 * Predictor: the right-hand side at level n is computed from the state with
 * ghosts at t^n and kept as history; w and U*, V* are advanced by the
 * third-order Adams-Bashforth formulas (15)-(17), the [F*]_t and [G*]_t terms
 * by the extrapolation 2F*^n - 3F*^{n-1} + F*^{n-2}.  During the first two
 * steps after a (re)start the history is incomplete and first-order Euler is
 * used (w += dt E^n, U* += dt F^n; the F*, G* increments are taken as zero
 * and no corrector runs).  P and Q are recovered from U*, V* by the
 * tridiagonal solves (21)-(22) with ghosts at t^{n+1}.
 * Corrector (iterated n_corr times): the right-hand side of the current
 * estimate (ghosts at t^{n+1}) enters the fourth-order Adams-Moulton formulas
 * (18)-(20), whose F*^p - F*^n term uses the F* of that estimate.
 * After each predictor/corrector solve the shoreline fix is applied; after
 * the last one the sponge layers damp eta, P, Q once per step (eq. 30). */
static void step_once(or_domain *D) {
    const int64_t s = D->step + 1; /* 1-based index of this step */
    const double dt = D->p.dt, t0 = D->t, t1 = D->t + D->p.dt;
    const size_t N = ncells_ghosted(D);
    const int n0 = (int)((s - 1) % 3), n1 = (int)((s + 1) % 3), n2 = (int)(s % 3);
    /* n0: level n, n1: level n-1, n2: level n-2 */
    double *U0 = calloc(N, sizeof(double)), *V0 = calloc(N, sizeof(double));
    double *w1 = calloc(N, sizeof(double)), *P1 = calloc(N, sizeof(double));
    double *Q1 = calloc(N, sizeof(double)), *U1 = calloc(N, sizeof(double));
    double *V1 = calloc(N, sizeof(double));
    double *Ek = calloc(N, sizeof(double)), *Fk = calloc(N, sizeof(double));
    double *Gk = calloc(N, sizeof(double)), *Fsk = calloc(N, sizeof(double));
    double *Gsk = calloc(N, sizeof(double));

    fill_ghosts(D, D->w, D->P, D->Q, t0);
    rhs(D, D->w, D->P, D->Q, D->E[n0], D->F[n0], D->G[n0], D->Fs[n0], D->Gs[n0]);
    ustar(D, D->P, D->Q, U0, V0);

    const double *E0 = D->E[n0], *E1 = D->E[n1], *E2 = D->E[n2];
    const double *F0 = D->F[n0], *F1 = D->F[n1], *F2 = D->F[n2];
    const double *G0 = D->G[n0], *G1 = D->G[n1], *G2 = D->G[n2];
    const double *Fs0 = D->Fs[n0], *Fs1 = D->Fs[n1], *Fs2 = D->Fs[n2];
    const double *Gs0 = D->Gs[n0], *Gs1 = D->Gs[n1], *Gs2 = D->Gs[n2];
    const int euler = s <= 2;
    /* predicted increment F*^{n+1} - F*^n: eq. (16) prints the quadratic
     * extrapolation 2F*^n - 3F*^{n-1} + F*^{n-2}; with a fixed number of
     * correctors that form is linearly unstable for two-dimensional flow once
     * d/dx exceeds about 4.5 (the paper's own runs use 6-26), so the default
     * is the linear extrapolation F*^n - F*^{n-1} (the corrector, eqs. 19-20,
     * is unchanged). */
    double x0 = 0.0, x1 = 0.0, x2 = 0.0;
    if (D->p.fstar_extrap == 2) { x0 = 2.0; x1 = -3.0; x2 = 1.0; }
    else if (D->p.fstar_extrap == 1) { x0 = 1.0; x1 = -1.0; }

#pragma omp parallel for schedule(static)
    for (int j = 0; j < D->p.ny; ++j)
        for (int i = 0; i < D->p.nx; ++i) {
            size_t c = CI(D, i, j);
            if (euler) {
                w1[c] = D->w[c] + dt * E0[c];
                U1[c] = U0[c] + dt * F0[c];
                V1[c] = V0[c] + dt * G0[c];
            } else {
                w1[c] = D->w[c] + dt / 12.0 * (23.0 * E0[c] - 16.0 * E1[c] + 5.0 * E2[c]);
                U1[c] = U0[c] + dt / 12.0 * (23.0 * F0[c] - 16.0 * F1[c] + 5.0 * F2[c]) +
                        x0 * Fs0[c] + x1 * Fs1[c] + x2 * Fs2[c];
                V1[c] = V0[c] + dt / 12.0 * (23.0 * G0[c] - 16.0 * G1[c] + 5.0 * G2[c]) +
                        x0 * Gs0[c] + x1 * Gs1[c] + x2 * Gs2[c];
            }
        }
    dry_fix_w(D, w1);
    solve_rows(D, U1, P1, t1);
    solve_cols(D, V1, Q1, t1);
    dry_fix_pq(D, w1, P1, Q1);

    /* with a tolerance set, the corrector is iterated until the largest
     * change of w and that of P, Q between two successive iterates (the
     * predictor's for the first) fall within it, at most n_corr times */
    const int conv = D->tol_w > 0.0;
    double *wp = NULL, *Pp = NULL, *Qp = NULL;
    if (conv) {
        wp = calloc(N, sizeof(double));
        Pp = calloc(N, sizeof(double));
        Qp = calloc(N, sizeof(double));
    }
    int ncorr = 0;
    if (!euler)
        for (int k = 0; k < D->p.n_corr; ++k) {
            if (conv) {
                memcpy(wp, w1, N * sizeof(double));
                memcpy(Pp, P1, N * sizeof(double));
                memcpy(Qp, Q1, N * sizeof(double));
            }
            fill_ghosts(D, w1, P1, Q1, t1);
            rhs(D, w1, P1, Q1, Ek, Fk, Gk, Fsk, Gsk);
#pragma omp parallel for schedule(static)
            for (int j = 0; j < D->p.ny; ++j)
                for (int i = 0; i < D->p.nx; ++i) {
                    size_t c = CI(D, i, j);
                    w1[c] = D->w[c] + dt / 24.0 * (9.0 * Ek[c] + 19.0 * E0[c] - 5.0 * E1[c] + E2[c]);
                    U1[c] = U0[c] + dt / 24.0 * (9.0 * Fk[c] + 19.0 * F0[c] - 5.0 * F1[c] + F2[c]) +
                            Fsk[c] - Fs0[c];
                    V1[c] = V0[c] + dt / 24.0 * (9.0 * Gk[c] + 19.0 * G0[c] - 5.0 * G1[c] + G2[c]) +
                            Gsk[c] - Gs0[c];
                }
            dry_fix_w(D, w1);
            solve_rows(D, U1, P1, t1);
            solve_cols(D, V1, Q1, t1);
            dry_fix_pq(D, w1, P1, Q1);
            ++ncorr;
            if (conv) {
                double dw = 0.0, dpq = 0.0;
                for (int j = 0; j < D->p.ny; ++j)
                    for (int i = 0; i < D->p.nx; ++i) {
                        size_t c = CI(D, i, j);
                        const double a = fabs(w1[c] - wp[c]);
                        const double b = fmax(fabs(P1[c] - Pp[c]), fabs(Q1[c] - Qp[c]));
                        dw = (a > dw || a != a) ? a : dw;       /* a NaN change never converges */
                        dpq = (b > dpq || b != b) ? b : dpq;
                    }
                D->last_dw = dw;
                D->last_dpq = dpq;
                if (dw <= D->tol_w && dpq <= D->tol_pq) break;
            }
        }
    D->last_corr = ncorr;
    D->total_corr += ncorr;
    free(wp); free(Pp); free(Qp);

    sponge(D, w1, P1, Q1);
    memcpy(D->w, w1, N * sizeof(double));
    memcpy(D->P, P1, N * sizeof(double));
    memcpy(D->Q, Q1, N * sizeof(double));
    D->step = s;
    D->t = t1;
    free(U0); free(V0); free(w1); free(P1); free(Q1); free(U1); free(V1);
    free(Ek); free(Fk); free(Gk); free(Fsk); free(Gsk);
}

/* ------------------------------------------------------------- C interface */
or_domain *or_create(const or_params *p, const double *z_corners) {
    if (!p || p->nx < 2 || p->ny < 2 || !(p->dx > 0) || !(p->dy > 0) || !(p->dt > 0)) return NULL;
    or_domain *D = calloc(1, sizeof(or_domain));
    D->p = *p;
    D->sx = p->nx + 4;
    D->zx = p->nx + 5;
    D->z = calloc((size_t)(p->nx + 5) * (size_t)(p->ny + 5), sizeof(double));
    for (int cj = 0; cj <= p->ny; ++cj)
        for (int ci = 0; ci <= p->nx; ++ci)
            D->z[ZI(D, ci, cj)] = z_corners[(size_t)cj * (p->nx + 1) + ci];
    size_t N = ncells_ghosted(D);
    D->w = calloc(N, sizeof(double));
    D->P = calloc(N, sizeof(double));
    D->Q = calloc(N, sizeof(double));
    for (int k = 0; k < 3; ++k) {
        D->E[k] = calloc(N, sizeof(double));
        D->F[k] = calloc(N, sizeof(double));
        D->G[k] = calloc(N, sizeof(double));
        D->Fs[k] = calloc(N, sizeof(double));
        D->Gs[k] = calloc(N, sizeof(double));
    }
    for (int s = 0; s < 4; ++s) D->side[s].type = OR_SOLID;
    fill_bathy_ghosts(D);
    /* lake at rest: w = max(w_s, bottom), no discharge */
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) D->w[CI(D, i, j)] = fmax(p->ws, bcell(D, i, j));
    return D;
}

void or_destroy(or_domain *D) {
    if (!D) return;
    free(D->z);
    free(D->w);
    free(D->P);
    free(D->Q);
    for (int k = 0; k < 3; ++k) {
        free(D->E[k]); free(D->F[k]); free(D->G[k]); free(D->Fs[k]); free(D->Gs[k]);
    }
    free(D);
}

/* Boundary type per side.  Wave-maker components (amplitude, period,
 * direction in radians, phase); their wave numbers follow eq. (29) at the
 * reference depth ref_depth, or, when ref_depth <= 0, at the mean still water
 * depth of the interior cells next to that side; c = omega / k (eq. 28). */
int or_set_boundary(or_domain *D, int side, int type, int width, int ncomp, const double *amp,
                    const double *period, const double *theta, const double *phase,
                    double ref_depth) {
    if (!D || side < 0 || side > 3 || type < 0 || type > 2 || ncomp < 0 || ncomp > OR_MAXC)
        return -1;
    or_side *s = &D->side[side];
    s->type = type;
    s->width = width;
    s->expo = 1.0;
    s->reflect = 0.0;
    s->ncomp = type == OR_WAVES ? ncomp : 0;
    fill_bathy_ghosts(D);
    double dref = ref_depth;
    if (!(dref > 0.0)) {
        double sum = 0.0;
        int n = 0;
        if (side == OR_WEST || side == OR_EAST) {
            int i = side == OR_WEST ? 0 : D->p.nx - 1;
            for (int j = 0; j < D->p.ny; ++j, ++n) sum += dstill(D, i, j);
        } else {
            int j = side == OR_SOUTH ? 0 : D->p.ny - 1;
            for (int i = 0; i < D->p.nx; ++i, ++n) sum += dstill(D, i, j);
        }
        dref = sum / n;
    }
    for (int m = 0; m < s->ncomp; ++m) {
        if (!(dref > 0.0) || !(period[m] > 0.0)) return -1;
        s->amp[m] = amp[m];
        s->omega[m] = 2.0 * M_PI / period[m];
        s->k[m] = or_eckart_k(s->omega[m], dref, D->p.g);
        s->c[m] = s->omega[m] / s->k[m];
        s->dirx[m] = cos(theta[m]);
        s->diry[m] = sin(theta[m]);
        s->phase[m] = phase ? phase[m] : 0.0;
    }
    return 0;
}

/* Corrector iteration until convergence (sec. 2.3): with tol_w > 0 every
 * full step iterates the corrector until max |w_k - w_{k-1}| <= tol_w and
 * max(|P_k - P_{k-1}|, |Q_k - Q_{k-1}|) <= tol_pq over the interior cells
 * (iterate 0 being the predictor's), at most n_corr times; the sponge
 * follows as always.  tol_w <= 0 restores the fixed count.  Resets the
 * counters of or_corrector_stats. */
int or_set_corrector_tolerance(or_domain *D, double tol_w, double tol_pq) {
    if (!D || tol_w != tol_w || tol_pq != tol_pq) return -1;
    D->tol_w = tol_w;
    D->tol_pq = tol_pq;
    D->last_corr = 0;
    D->total_corr = 0;
    D->last_dw = D->last_dpq = 0.0;
    return 0;
}

/* Change parameters of a running domain (sec. 3.3: the user may alter the
 * physical and numerical parameters while the model runs).  nx, ny, dx, dy,
 * n_corr and ws must stay; a new dt restarts the multistep history (the step
 * count restarts from 0, so the next two steps are Euler steps of sec. 2.3;
 * the time goes on) and rescales partially reflective sponges; the state is
 * kept.  A new model or B that leaves eq. (23) without diagonal dominance is
 * refused (-2) with the domain unchanged. */
int or_diag_dominant(const or_domain *D);
int or_set_sponge_reflect(or_domain *D, int side, double R);

int or_update_params(or_domain *D, const or_params *p) {
    if (!D || !p) return -1;
    const or_params o = D->p;
    if (p->nx != o.nx || p->ny != o.ny || p->dx != o.dx || p->dy != o.dy || p->n_corr != o.n_corr ||
        p->ws != o.ws || !(p->dt > 0) || !(p->g > 0) || !(p->theta >= 1.0 && p->theta <= 2.0) || !(p->eps > 0) ||
        (p->model != OR_BSNQ && p->model != OR_NLSW) || p->friction < 0 || p->friction > 2 ||
        p->fstar_extrap < 0 || p->fstar_extrap > 2 || !(p->Bdisp >= 0) || !(p->fcoef >= 0))
        return -1;
    D->p = *p;
    if (!or_diag_dominant(D)) {
        D->p = o;
        return -2;
    }
    if (p->dt != o.dt) {
        D->step = 0;
        for (int q = 0; q < 4; ++q)
            if (D->side[q].type == OR_SPONGE && D->side[q].reflect > 0.0)
                or_set_sponge_reflect(D, q, D->side[q].reflect);
    }
    return 0;
}

/* Corrector count of the following steps (fixed-count mode; the cap in the
 * tolerance mode). */
int or_set_n_corr(or_domain *D, int n_corr) {
    if (!D || n_corr < 0) return -1;
    D->p.n_corr = n_corr;
    return 0;
}

/* Correctors of the last step and since the tolerance was set; the changes
 * measured after the last corrector (tolerance mode only). */
int or_corrector_stats(const or_domain *D, int *last, int64_t *total, double *dw, double *dpq) {
    if (!D) return -1;
    if (last) *last = D->last_corr;
    if (total) *total = D->total_corr;
    if (dw) *dw = D->last_dw;
    if (dpq) *dpq = D->last_dpq;
    return 0;
}

/* Partially reflective sponge (the paper names such layers without giving a
 * formula).  The layer multiplies eta, P, Q by gamma^s each step.  A long
 * wave of speed c = sqrt(g d) that crosses the layer of width L and comes
 * back spends 2 / (c dt) steps per unit of distance in it, so its amplitude
 * changes by the factor exp(s (2 / (c dt)) int_0^L ln gamma dD); with
 * gamma = cos^2(pi (L - D) / (2L)) of eq. (30) the integral is -2 L ln 2, and
 * the factor exp(-4 s L ln 2 / (c dt)).  A target reflection coefficient R
 * in (0, 1) thus gives s = -ln(R) c dt / (4 L ln 2), capped at 1 (the layer
 * of eq. 30 itself, which reflects less than such an R); R = 0 keeps s = 1
 * and R = 1 gives s = 0, a solid wall.  d: mean still water depth of the
 * interior cells next to the side, dry cells counting 0 (s = 1 where the
 * mean is not positive).  The side must be a sponge; set after
 * or_set_boundary. */
int or_set_sponge_reflect(or_domain *D, int side, double R) {
    if (!D || side < 0 || side > 3 || D->side[side].type != OR_SPONGE || !(R >= 0.0 && R <= 1.0)) return -1;
    or_side *s = &D->side[side];
    s->reflect = R;
    if (R == 0.0) {
        s->expo = 1.0;
    s->reflect = 0.0;
        return 0;
    }
    if (R == 1.0) {
        s->expo = 0.0;
        return 0;
    }
    double sum = 0.0;
    int n = 0;
    if (side == OR_WEST || side == OR_EAST) {
        int i = side == OR_WEST ? 0 : D->p.nx - 1;
        for (int j = 0; j < D->p.ny; ++j, ++n) sum += fmax(dstill(D, i, j), 0.0);
    } else {
        int j = side == OR_SOUTH ? 0 : D->p.ny - 1;
        for (int i = 0; i < D->p.nx; ++i, ++n) sum += fmax(dstill(D, i, j), 0.0);
    }
    const double d = sum / n;  /* dry cells count as depth 0 */
    const double L = s->width * (side == OR_WEST || side == OR_EAST ? D->p.dx : D->p.dy);
    if (!(d > 0.0)) {
        s->expo = 1.0;
    s->reflect = 0.0;
        return 0;
    }
    const double e = -log(R) * sqrt(D->p.g * d) * D->p.dt / (4.0 * L * log(2.0));
    s->expo = e < 1.0 ? e : 1.0;
    return 0;
}

/* Hot start (sec. 3.2): set w, P, Q (interior, row-major nx*ny) and the time;
 * the multistep history restarts with the Euler steps. */
int or_set_state(or_domain *D, const double *w, const double *P, const double *Q, double t) {
    for (int j = 0; j < D->p.ny; ++j)
        for (int i = 0; i < D->p.nx; ++i) {
            size_t k = (size_t)j * D->p.nx + i, c = CI(D, i, j);
            D->w[c] = w[k];
            D->P[c] = P[k];
            D->Q[c] = Q[k];
        }
    D->t = t;
    D->step = 0;
    D->health = 0;
    return 0;
}

int or_get_state(const or_domain *D, double *w, double *P, double *Q) {
    for (int j = 0; j < D->p.ny; ++j)
        for (int i = 0; i < D->p.nx; ++i) {
            size_t k = (size_t)j * D->p.nx + i, c = CI(D, i, j);
            if (w) w[k] = D->w[c];
            if (P) P[k] = D->P[c];
            if (Q) Q[k] = D->Q[c];
        }
    return 0;
}

/* Cell bottom and still water depth, interior, row-major. */
int or_get_bathy(const or_domain *D, double *bottom, double *depth) {
    for (int j = 0; j < D->p.ny; ++j)
        for (int i = 0; i < D->p.nx; ++i) {
            size_t k = (size_t)j * D->p.nx + i;
            if (bottom) bottom[k] = bcell(D, i, j);
            if (depth) depth[k] = dstill(D, i, j);
        }
    return 0;
}

/* Bilinear bottom at a point (x, y) inside the domain. */
static double bottom_at(const or_domain *D, double x, double y) {
    double fx = x / D->p.dx, fy = y / D->p.dy;
    int ci = (int)floor(fx), cj = (int)floor(fy);
    if (ci < 0) ci = 0;
    if (ci > D->p.nx - 1) ci = D->p.nx - 1;
    if (cj < 0) cj = 0;
    if (cj > D->p.ny - 1) cj = D->p.ny - 1;
    double ax = fx - ci, ay = fy - cj;
    return (1 - ax) * (1 - ay) * zc(D, ci, cj) + ax * (1 - ay) * zc(D, ci + 1, cj) +
           (1 - ax) * ay * zc(D, ci, cj + 1) + ax * ay * zc(D, ci + 1, cj + 1);
}

/* Superpose a solitary wave, sec. 2.7, eqs. (33)-(36): height H, direction
 * theta, crest through (x0, y0); d is the still water depth at the crest
 * point; added only in cells with d > 0. */
int or_add_solitary(or_domain *D, double H, double theta, double x0, double y0) {
    double d = D->p.ws - bottom_at(D, x0, y0);
    if (!(d > 0.0) || !(H + d > 0.0)) return -1;
    double ks = sqrt(3.0 * fabs(H) / (4.0 * d * d * d));
    double cs = sqrt(D->p.g * (H + d));
    double ct = cos(theta), st = sin(theta);
    for (int j = 0; j < D->p.ny; ++j)
        for (int i = 0; i < D->p.nx; ++i) {
            if (dstill(D, i, j) <= 0.0) continue;
            double x = (i + 0.5) * D->p.dx, y = (j + 0.5) * D->p.dy;
            double sech = 1.0 / cosh(ks * ((x - x0) * ct + (y - y0) * st));
            double eta = H * sech * sech;
            size_t c = CI(D, i, j);
            D->w[c] += eta;
            D->P[c] += cs * eta * ct;
            D->Q[c] += cs * eta * st;
        }
    return 0;
}

/* Diagonal dominance of every row and column system (eq. 23): required for
 * the solves without pivoting. */
int or_diag_dominant(const or_domain *D) {
    for (int j = 0; j < D->p.ny; ++j)
        for (int i = 0; i < D->p.nx; ++i) {
            double A, Bm, C;
            row_coefs(D, i, j, &A, &Bm, &C);
            if (!(fabs(Bm) > fabs(A) + fabs(C))) return 0;
            col_coefs(D, i, j, &A, &Bm, &C);
            if (!(fabs(Bm) > fabs(A) + fabs(C))) return 0;
        }
    return 1;
}

/* Interactive edits (sec. 1): a Gaussian hump exp(-r^2 / (2 sigma^2)) of
 * amplitude amp added to the water surface (kind 0) or to the terrain corners
 * (kind 1).  The surface never ends below the bottom; the history is kept. */
int or_apply_edit(or_domain *D, int kind, double x0, double y0, double amp, double sigma) {
    if (!(sigma > 0.0) || (kind != OR_EDIT_WATER && kind != OR_EDIT_TERRAIN)) return -1;
    if (kind == OR_EDIT_WATER) {
        for (int j = 0; j < D->p.ny; ++j)
            for (int i = 0; i < D->p.nx; ++i) {
                double x = (i + 0.5) * D->p.dx - x0, y = (j + 0.5) * D->p.dy - y0;
                D->w[CI(D, i, j)] += amp * exp(-(x * x + y * y) / (2.0 * sigma * sigma));
            }
    } else {
        /* Terrain change under water keeps the free surface and the
         * depth-averaged velocity (momentum scales with the remaining depth,
         * never up); the paper leaves the state's treatment open. */
        size_t nz = (size_t)(D->p.nx + 5) * (D->p.ny + 5);
        size_t nc = (size_t)D->p.nx * D->p.ny;
        double *save = malloc(nz * sizeof(double));
        double *hold = malloc(nc * sizeof(double));
        memcpy(save, D->z, nz * sizeof(double));
        for (int j = 0; j < D->p.ny; ++j)
            for (int i = 0; i < D->p.nx; ++i) hold[(size_t)j * D->p.nx + i] = D->w[CI(D, i, j)] - bcell(D, i, j);
        for (int cj = 0; cj <= D->p.ny; ++cj)
            for (int ci = 0; ci <= D->p.nx; ++ci) {
                double x = ci * D->p.dx - x0, y = cj * D->p.dy - y0;
                D->z[ZI(D, ci, cj)] += amp * exp(-(x * x + y * y) / (2.0 * sigma * sigma));
            }
        fill_bathy_ghosts(D);
        if (!or_diag_dominant(D)) {
            memcpy(D->z, save, nz * sizeof(double));
            free(save);
            free(hold);
            return -4;
        }
        for (int j = 0; j < D->p.ny; ++j)
            for (int i = 0; i < D->p.nx; ++i) {
                double ho = hold[(size_t)j * D->p.nx + i], hn = D->w[CI(D, i, j)] - bcell(D, i, j);
                if (hn < 0.0) hn = 0.0;
                double f = ho > 0.0 ? hn / ho : 1.0;
                if (f > 1.0) f = 1.0;
                D->P[CI(D, i, j)] *= f;
                D->Q[CI(D, i, j)] *= f;
            }
        free(save);
        free(hold);
    }
    dry_fix_w(D, D->w);
    dry_fix_pq(D, D->w, D->P, D->Q);
    return 0;
}

int or_advance(or_domain *D, int64_t nsteps) {
    for (int64_t k = 0; k < nsteps; ++k) step_once(D);
    check_health(D);
    return D->health ? -5 : 0;
}

int64_t or_get_step(const or_domain *D) { return D->step; }
double or_get_time(const or_domain *D) { return D->t; }

/* ---------------------------------------------------------- test access */
/* Right-hand side (E, F, G, F*, G*) and (U*, V*) of an interior state (w, P,
 * Q, row-major nx*ny) with ghosts at time t, written row-major. */
int or_eval_rhs(or_domain *D, const double *w, const double *P, const double *Q, double t,
                double *E, double *F, double *G, double *Fs, double *Gs, double *U, double *V) {
    size_t N = ncells_ghosted(D);
    double *a[8];
    for (int k = 0; k < 8; ++k) a[k] = calloc(N, sizeof(double));
    for (int j = 0; j < D->p.ny; ++j)
        for (int i = 0; i < D->p.nx; ++i) {
            size_t k = (size_t)j * D->p.nx + i, c = CI(D, i, j);
            a[0][c] = w[k];
            a[1][c] = P[k];
            a[2][c] = Q[k];
        }
    fill_ghosts(D, a[0], a[1], a[2], t);
    rhs(D, a[0], a[1], a[2], a[3], a[4], a[5], a[6], a[7]);
    double *Ub = calloc(N, sizeof(double)), *Vb = calloc(N, sizeof(double));
    ustar(D, a[1], a[2], Ub, Vb);
    double *outs[7] = {E, F, G, Fs, Gs, U, V};
    double *srcs[7] = {a[3], a[4], a[5], a[6], a[7], Ub, Vb};
    for (int o = 0; o < 7; ++o) {
        if (!outs[o]) continue;
        for (int j = 0; j < D->p.ny; ++j)
            for (int i = 0; i < D->p.nx; ++i)
                outs[o][(size_t)j * D->p.nx + i] = srcs[o][CI(D, i, j)];
    }
    for (int k = 0; k < 8; ++k) free(a[k]);
    free(Ub);
    free(Vb);
    return 0;
}

/* Threads of the OpenMP row/column loops for the following calls (n <= 0:
 * leave unchanged); returns the number now in use.  Results do not depend
 * on it. */
int or_set_threads(int n) {
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}

/* Set the number of completed steps and the time.  Together with
 * or_set_history it lets a step start from a known multistep history instead
 * of the Euler start-up of sec. 2.3 (steps 1 and 2 after a start). */
int or_set_clock(or_domain *D, int64_t step, double t) {
    if (step < 0) return -1;
    D->step = step;
    D->t = t;
    return 0;
}

/* Load the right-hand side (E, F, G, F*, G*) of an earlier time level into
 * the multistep history ring: lag 1 is level n-1 and lag 2 level n-2 with
 * respect to the next step (whose own level n its predictor computes).
 * Arrays are interior, row-major nx*ny; a NULL array loads zeros. */
int or_set_history(or_domain *D, int lag, const double *E, const double *F, const double *G,
                   const double *Fs, const double *Gs) {
    if (lag < 1 || lag > 2) return -1;
    const int slot = (int)(((D->step - lag) % 3 + 3) % 3);
    const double *src[5] = {E, F, G, Fs, Gs};
    double *dst[5] = {D->E[slot], D->F[slot], D->G[slot], D->Fs[slot], D->Gs[slot]};
    for (int f = 0; f < 5; ++f)
        for (int j = 0; j < D->p.ny; ++j)
            for (int i = 0; i < D->p.nx; ++i)
                dst[f][CI(D, i, j)] = src[f] ? src[f][(size_t)j * D->p.nx + i] : 0.0;
    return 0;
}

/* Solve the row systems (21) and column systems (22) for right-hand sides
 * U, V (interior, row-major) with wave-maker ghosts at time t. */
int or_eval_solve(or_domain *D, const double *U, const double *V, double t, double *P, double *Q) {
    size_t N = ncells_ghosted(D);
    double *Ub = calloc(N, sizeof(double)), *Vb = calloc(N, sizeof(double));
    double *Pb = calloc(N, sizeof(double)), *Qb = calloc(N, sizeof(double));
    for (int j = 0; j < D->p.ny; ++j)
        for (int i = 0; i < D->p.nx; ++i) {
            Ub[CI(D, i, j)] = U[(size_t)j * D->p.nx + i];
            Vb[CI(D, i, j)] = V[(size_t)j * D->p.nx + i];
        }
    solve_rows(D, Ub, Pb, t);
    solve_cols(D, Vb, Qb, t);
    for (int j = 0; j < D->p.ny; ++j)
        for (int i = 0; i < D->p.nx; ++i) {
            P[(size_t)j * D->p.nx + i] = Pb[CI(D, i, j)];
            Q[(size_t)j * D->p.nx + i] = Qb[CI(D, i, j)];
        }
    free(Ub); free(Vb); free(Pb); free(Qb);
    return 0;
}

/* Reconstruction of one cell along one direction (steps 1-2 of sec. 2.2):
 * inputs (w, n, t) at the previous, this and the next cell and the bottom at
 * the cell's low and high faces; output (w, n, t) at the low face then the
 * high face. */
void or_reconstruct(const double w[3], const double n[3], const double t[3], double b_lo,
                    double b_hi, double theta, double out[6]) {
    face_state lo, hi;
    reconstruct(w[0], w[1], w[2], n[0], n[1], n[2], t[0], t[1], t[2], b_lo, b_hi, theta, &lo, &hi);
    out[0] = lo.w; out[1] = lo.n; out[2] = lo.t;
    out[3] = hi.w; out[4] = hi.n; out[5] = hi.t;
}
