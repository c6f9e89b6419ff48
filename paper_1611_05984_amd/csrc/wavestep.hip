// wavestep.hip -- host side of the gfx950 time step: workspace layout, the
// C ABI of include/wavestep.h, and the launch sequence of one step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/wavestep.h"
#include "ws_batch.hpp"

using namespace ws;

// ------------------------------------------------------------ error handling
static thread_local std::string g_err;

static ws_status fail(ws_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIPCHK(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess)                                                              \
            return fail(WS_EHIP, "%s: %s (%s:%d)", #x, hipGetErrorString(e_), __FILE__, __LINE__); \
    } while (0)

extern "C" const char *ws_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------------ domain
struct ws_domain {
    ws_grid g;
    int nxp, nyp, pitch, zpitch, nu, nv;
    char *base;
    size_t bytes;
    float *D, *Dnew;               // corner still-water depth (+ scratch for terrain edits)
    float *st[3][3];               // state of the step and two estimates (eta, P, Q)
    float *rx, *ry;                // U*, V* increments / eliminated segments
    float *S[3];                   // corrector bases
    float *hist[3][5];             // [slot][E, F, G, F*, G*]
    float4 *redx, *redy;
    float *solx, *soly;
    float *lux, *luy;              // static factors of the reduced systems (factored solves)
    bool lu_valid;
    int lu_kind;                   // solver the factors were computed for
    float *ghost[2];               // wave-maker ghosts at t^n, t^{n+1}
    int gl;                        // ghost positions per layer
    double *tab[4];                // wave tables
    int *health;
    double *scal;                  // small device scratch (reductions)
    int side_type[4], side_width[4], side_ncomp[4];
    float side_expo[4];   // sponge damping exponent (1 = the layer of eq. 30)
    double side_R[4], side_depth[4];  // sponge target reflection and mean side depth it was set with
    int cur;
    int64_t step;
    double t;
    bool prof_on;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof;  // (class, start, stop)
    ws_batch *batch;               // batch this domain is attached to, if any
    int bidx;                      // its index in the batch's device tables
    bool stale;                    // the batch has advanced it since the last ws_batch_sync
    int64_t stop;                  // batch step limit (-1: none)
    int bhealth;                   // health word as of the last batch sync
    bool vdirty;                   // pass argument tables must be rewritten
    int sy, pnt, solver;           // tuning: stencil rows per strip, PCR threads per system, reduced solver
    int syc;                       // stencil rows per strip in corrector passes (0: sy)
    size_t fstride;                // bytes between consecutive fields
    StencilArgs *vsa;              // pass argument tables (device), batch use only
    SolveArgs *vso;
    int nvar;
    double tol_w, tol_pq;          // corrector iteration until convergence: off while tol_w <= 0
    int last_corr;                 // correctors the last step ran
    int64_t total_corr;            // correctors since the tolerance was set
    double last_dw, last_dpq;      // changes measured after the last corrector
    int static_dev;                // device whose static array holds the workspace (-1: the caller's)
};

static ws_status busy_check(const ws_domain *d, const char *who) {
    if (d->batch && d->stale) return fail(WS_EBUSY, "%s: domain advanced by its batch; call ws_batch_sync first", who);
    return WS_OK;
}
static void batch_touch(ws_domain *d);

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
static int roundup(int x, int m) { return (x + m - 1) / m * m; }

struct Layout {
    int nxp, nyp, pitch, zpitch, nu, nv, gl;
    size_t field, corners, redx, redy, solx, soly, lux, luy, ghost, tabs, misc, vtab, total;
    int nvar;
};

// The stencil addresses the fields of a group (up to five, one field stride
// apart) by 32-bit byte offsets from the group's base: five padded fields
// must span less than 4 GiB (about 2.1e8 cells; squares up to 14640 x 14640).
static bool offsets_fit(const ws_grid *g) {
    if (g->nx > (1 << 20) || g->ny > (1 << 20)) return false;
    const size_t field = align256(sizeof(float) * (size_t)roundup(g->ny, TY) * (size_t)roundup(g->nx, TX));
    return 5 * field <= 0xFFFFFFFFull;
}

static bool grid_ok(const ws_grid *g) {
    return g && g->nx >= 2 && g->ny >= 2 && offsets_fit(g) && g->dx > 0 && g->dy > 0 && g->dt > 0 && g->g > 0 &&
           g->n_corr >= 0 && g->n_corr <= 64 && (g->model == WS_BSNQ || g->model == WS_NLSW) &&
           g->friction >= 0 && g->friction <= 2 && g->fstar_extrap >= 0 && g->fstar_extrap <= 2 &&
           g->theta >= 1.0 && g->theta <= 2.0 && g->eps > 0;
}

static Layout layout(const ws_grid *g) {
    Layout L;
    L.nxp = roundup(g->nx, TX);
    L.nyp = roundup(g->ny, TY);
    L.pitch = L.nxp;
    L.zpitch = roundup(g->nx + 1, 64);
    L.nu = 2 * (L.nxp / MX);
    L.nv = 2 * (L.nyp / TY);
    L.gl = (g->nx > g->ny ? g->nx : g->ny) + 4;
    L.field = align256(sizeof(float) * (size_t)L.nyp * L.pitch);
    L.corners = align256(sizeof(float) * (size_t)(g->ny + 1) * L.zpitch);
    L.redx = align256(sizeof(float4) * (size_t)L.nyp * L.nu);
    L.redy = align256(sizeof(float4) * (size_t)L.nxp * L.nv);
    L.solx = align256(sizeof(float) * (size_t)L.nyp * L.nu);
    L.soly = align256(sizeof(float) * (size_t)L.nxp * L.nv);
    L.lux = align256(3 * sizeof(float) * (size_t)L.nyp * L.nu);
    L.luy = align256(3 * sizeof(float) * (size_t)L.nxp * L.nv);
    L.ghost = align256(sizeof(float) * 4 * 2 * 3 * (size_t)L.gl);
    L.tabs = align256(sizeof(double) * MAXC * TABW);
    L.misc = 256;
    // pass argument tables for batched stepping: 9 Euler start-up variants
    // (state buffer x step mod 3) and 9 x (n_corr + 1) passes of full steps
    L.nvar = 9 * (g->n_corr + 2);
    L.vtab = align256(L.nvar * (sizeof(StencilArgs) + sizeof(SolveArgs)));
    L.total = 29 * L.field + 2 * L.corners + L.redx + L.redy + L.solx + L.soly + L.lux + L.luy + 2 * L.ghost +
              4 * L.tabs + L.misc + L.vtab;
    return L;
}

extern "C" void ws_grid_defaults(ws_grid *g, int32_t nx, int32_t ny) {
    std::memset(g, 0, sizeof *g);
    g->nx = nx;
    g->ny = ny;
    g->n_corr = 2;
    g->model = WS_BSNQ;
    g->friction = WS_FRIC_NONE;
    g->fstar_extrap = 1;
    g->g = 9.81;
    g->still_water = 0.0;
    g->Bcoef = 1.0 / 15.0;
    g->theta = 1.3;
    g->eps = 5e-12;
    g->friction_coef = 0.0;
}

extern "C" size_t ws_workspace_bytes(const ws_grid *g) {
    if (!grid_ok(g)) return 0;
    return layout(g).total;
}

static Dom make_dom(const ws_domain *d) {
    Dom m;
    m.nx = d->g.nx;
    m.ny = d->g.ny;
    m.pitch = d->pitch;
    m.zpitch = d->zpitch;
    m.nu = d->nu;
    m.nv = d->nv;
    m.model = d->g.model;
    m.friction = d->g.friction;
    m.gl = d->gl;
    m.gh = d->ghost[0];
    m.dx = (float)d->g.dx;
    m.dy = (float)d->g.dy;
    m.rdx = (float)(1.0 / d->g.dx);
    m.rdy = (float)(1.0 / d->g.dy);
    m.g = (float)d->g.g;
    m.Bd = (float)d->g.Bcoef;
    m.theta = (float)d->g.theta;
    m.eps = (float)d->g.eps;
    m.fcoef = (float)d->g.friction_coef;
    m.D = d->D;
    for (int s = 0; s < 4; ++s) {
        m.side[s].type = d->side_type[s];
        m.side[s].width = d->side_width[s];
        m.side[s].ncomp = d->side_ncomp[s];
        m.side[s].expo = d->side_expo[s];
        m.side[s].tab = d->tab[s];
    }
    return m;
}

static dim3 tiles(const ws_domain *d) { return dim3(d->nxp / TX, d->nyp / TY); }

// ----------------------------------------------------------- small kernels
__global__ void k_corners_from_z(const float *z, float *D, int nx, int ny, int zpitch, float ws) {
    int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i <= nx && j <= ny) D[(size_t)j * zpitch + i] = ws - z[(size_t)j * (nx + 1) + i];
}

__device__ __forceinline__ float cell_Dc(const Dom &d, int i, int j) {
    const float *r0 = d.D + (size_t)j * d.zpitch, *r1 = r0 + d.zpitch;
    return 0.25f * ((r0[i] + r0[i + 1]) + (r1[i] + r1[i + 1]));
}

// Lake at rest: eta = max(0, -D_cell) (surface at still water or on the bottom).
__global__ void k_rest_state(Dom d, float *e, float *p, float *q) {
    int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    size_t o = (size_t)j * d.pitch + i;
    e[o] = fmaxf(0.f, -cell_Dc(d, i, j));
    p[o] = 0.f;
    q[o] = 0.f;
}

__global__ void k_set_state(Dom d, const float *w, const float *P, const float *Q, int ipitch,
                            float ws, float *e, float *p, float *q) {
    int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    size_t o = (size_t)j * d.pitch + i, s = (size_t)j * ipitch + i;
    e[o] = w[s] - ws;
    p[o] = P[s];
    q[o] = Q[s];
}

__global__ void k_read(Dom d, const float *e, const float *p, const float *q, int what, float ws,
                       float *first, float *P, float *Q, int opitch) {
    int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    size_t o = (size_t)j * d.pitch + i, s = (size_t)j * opitch + i;
    if (first) first[s] = what == WS_READ_H ? e[o] + cell_Dc(d, i, j) : e[o] + ws;
    if (P) P[s] = p[o];
    if (Q) Q[s] = q[o];
}

// Gauges: the state at chosen cells.  Gauge k at cell (ij[2k], ij[2k+1])
// gives out[4k..4k+3] = (w, h, P, Q); a cell outside the grid gives NaNs.
__global__ void k_gauges(Dom d, const float *e, const float *p, const float *q, float ws, const int *ij, int n,
                         float *out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int i = ij[2 * k], j = ij[2 * k + 1];
    float v0 = NAN, v1 = NAN, v2 = NAN, v3 = NAN;
    if (i >= 0 && i < d.nx && j >= 0 && j < d.ny) {
        const size_t o = (size_t)j * d.pitch + i;
        v0 = e[o] + ws;
        v1 = e[o] + cell_Dc(d, i, j);
        v2 = p[o];
        v3 = q[o];
    }
    out[4 * k] = v0;
    out[4 * k + 1] = v1;
    out[4 * k + 2] = v2;
    out[4 * k + 3] = v3;
}

// Surface kept at or above the bottom, discharges desingularized where thin.
__device__ __forceinline__ void shore_fix(const Dom &d, int i, int j, float *e, float *p, float *q) {
    size_t o = (size_t)j * d.pitch + i;
    float Dc = cell_Dc(d, i, j);
    float ev = fmaxf(e[o], -Dc);
    e[o] = ev;
    float h = ev + Dc, h2 = h * h, h4 = h2 * h2;
    if (h4 < d.eps) {
        float f = 1.41421356237f * h2 * rsqrtf(h4 + d.eps);
        p[o] *= f;
        q[o] *= f;
    }
}

__global__ void k_solitary(Dom d, float *e, float *p, float *q, double H, double ks, double cs,
                           double ct, double st, double x0, double y0) {
    int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    if (!(cell_Dc(d, i, j) > 0.f)) return;
    double x = (i + 0.5) * d.dx, y = (j + 0.5) * d.dy;
    double sc = 1.0 / cosh(ks * ((x - x0) * ct + (y - y0) * st));
    double eta = H * sc * sc;
    size_t o = (size_t)j * d.pitch + i;
    e[o] += (float)eta;
    p[o] += (float)(cs * eta * ct);
    q[o] += (float)(cs * eta * st);
}

__global__ void k_edit_water(Dom d, float *e, float *p, float *q, double x0, double y0, double amp,
                             double sigma) {
    int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    double x = (i + 0.5) * d.dx - x0, y = (j + 0.5) * d.dy - y0;
    size_t o = (size_t)j * d.pitch + i;
    e[o] += (float)(amp * exp(-(x * x + y * y) / (2.0 * sigma * sigma)));
    shore_fix(d, i, j, e, p, q);
}

__global__ void k_edit_terrain(Dom d, const float *Dold, float *Dnew, double x0, double y0,
                               double amp, double sigma) {
    int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i > d.nx || j > d.ny) return;
    double x = i * (double)d.dx - x0, y = j * (double)d.dy - y0;
    size_t o = (size_t)j * d.zpitch + i;
    Dnew[o] = (float)((double)Dold[o] - amp * exp(-(x * x + y * y) / (2.0 * sigma * sigma)));
}

// After a terrain change (d holds the new depth, Dold the old one): the
// surface is kept and the momentum scaled by remaining / old depth (at most
// 1), which keeps the depth-averaged velocity of cells that stay wet.
__global__ void k_edit_velocity(Dom d, const float *Dold, const float *e, float *p, float *q) {
    int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    Dom od = d;
    od.D = Dold;
    const size_t o = (size_t)j * d.pitch + i;
    const float ho = e[o] + cell_Dc(od, i, j), hn = fmaxf(e[o] + cell_Dc(d, i, j), 0.f);
    const float f = ho > 0.f ? fminf(hn / ho, 1.f) : 1.f;
    p[o] *= f;
    q[o] *= f;
}
__global__ void k_shore_fix(Dom d, float *e, float *p, float *q) {
    int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    shore_fix(d, i, j, e, p, q);
}

// Diagonal dominance of every row and column system (raw coefficients of eq. 23).
__global__ void k_check_dd(Dom d, int *flag) {
    int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    auto dcell = [&](int a, int b) {
        return fmaxf(0.25f * ((corner_D(d, a, b) + corner_D(d, a + 1, b)) +
                              (corner_D(d, a, b + 1) + corner_D(d, a + 1, b + 1))), 0.f);
    };
    const float dc = dcell(i, j);
    float A, B, C;
    tri_coef(d, tri_k(d.Bd, d.rdx), dc, dcell(i + 1, j) - dcell(i - 1, j), A, B, C);
    bool bad = !(fabsf(B) > fabsf(A) + fabsf(C));
    tri_coef(d, tri_k(d.Bd, d.rdy), dc, dcell(i, j + 1) - dcell(i, j - 1), A, B, C);
    bad |= !(fabsf(B) > fabsf(A) + fabsf(C));
    if (bad) atomicOr(flag, 1);
}

// Mean still-water depth of the first interior row/column along a side.
__global__ void k_side_depth(Dom d, int side, double *out) {
    __shared__ double part[256];
    const bool xs = side < 2;
    const int n = xs ? d.ny : d.nx;
    double s = 0.0;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        int i = xs ? (side == 0 ? 0 : d.nx - 1) : k;
        int j = xs ? k : (side == 2 ? 0 : d.ny - 1);
        s += fmaxf(cell_Dc(d, i, j), 0.f);
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = part[0] / n;
}

static dim3 cells_grid(int nx, int ny) { return dim3((nx + 255) / 256, ny); }

// Largest change between two iterates of the state over the interior cells:
// res[0] = max |eta1 - eta0|, res[1] = max(|P1 - P0|, |Q1 - Q0|), kept as
// float bits (non-negative floats order as unsigned integers); a non-finite
// change counts as +inf.
__device__ __forceinline__ float change(float a, float b) {
    const float c = fabsf(a - b);
    return isfinite(c) ? c : INFINITY;
}
__global__ void k_residual(Dom d, const float *e0, const float *p0, const float *q0, const float *e1, const float *p1,
                           const float *q1, unsigned *res) {
    float mw = 0.f, mq = 0.f;
    const int n = d.nx * d.ny;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        const int j = k / d.nx, i = k - j * d.nx;
        const size_t o = (size_t)j * d.pitch + i;
        mw = fmaxf(mw, change(e1[o], e0[o]));
        mq = fmaxf(mq, fmaxf(change(p1[o], p0[o]), change(q1[o], q0[o])));
    }
    for (int off = 32; off > 0; off >>= 1) {
        mw = fmaxf(mw, __shfl_xor(mw, off));
        mq = fmaxf(mq, __shfl_xor(mq, off));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&res[0], __float_as_uint(mw));
        atomicMax(&res[1], __float_as_uint(mq));
    }
}
__global__ void k_zero_words(unsigned *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// The sponge of the step's end as a pass of its own (the same arithmetic as
// the last expand's epilogue, which applies it when the corrector count is
// fixed): eta, P, Q times the layers' factors where the still water depth is
// positive.
__global__ void k_sponge(Dom d, float *e, float *P, float *Q) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    const float *r0 = d.D + (size_t)j * d.zpitch, *r1 = r0 + d.zpitch;
    const float Dc = 0.25f * ((r0[i] + r0[i + 1]) + (r1[i] + r1[i + 1]));
    if (!(Dc > 0.f)) return;
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
        const size_t o = (size_t)j * d.pitch + i;
        e[o] *= gm;
        P[o] *= gm;
        Q[o] *= gm;
    }
}

// ------------------------------------------------------------------ API
// Argument checks shared by both ways of creating a domain.
static ws_status init_checks(const ws_grid *g, const float *z_corners_dev, const void *workspace_dev,
                             size_t workspace_bytes, const char *who) {
    if (!grid_ok(g)) return fail(WS_EINVAL, "%s: invalid grid parameters", who);
    if (!z_corners_dev || !workspace_dev) return fail(WS_EINVAL, "%s: NULL device pointer", who);
    if (((uintptr_t)workspace_dev & 255) != 0) return fail(WS_EINVAL, "%s: workspace not 256-byte aligned", who);
    Layout L = layout(g);
    if (L.nu > NRED_MAX || L.nv > NRED_MAX) return fail(WS_EINVAL, "%s: grid too large (max %d x %d)", who, NRED_MAX / 2 * MX, NRED_MAX / 2 * TY);
    if (workspace_bytes < L.total) return fail(WS_ENOMEM, "%s: workspace %zu < %zu bytes", who, workspace_bytes, L.total);
    return WS_OK;
}

// Lay the domain's fields out in the workspace, clear it, load the bathymetry
// and the lake at rest, and check diagonal dominance.  `d` is a freshly
// constructed handle; on failure the caller disposes of it.
static ws_status domain_setup(ws_domain *d, const ws_grid *g, const float *z_corners_dev, void *workspace_dev,
                              size_t workspace_bytes, void *stream, const char *who) {
    Layout L = layout(g);
    d->g = *g;
    d->static_dev = -1;
    d->nxp = L.nxp; d->nyp = L.nyp; d->pitch = L.pitch; d->zpitch = L.zpitch; d->nu = L.nu; d->nv = L.nv;
    d->gl = L.gl;
    d->base = (char *)workspace_dev;
    d->bytes = workspace_bytes;
    char *p = d->base;
    auto take = [&](size_t n) { char *r = p; p += n; return r; };
    for (int b = 0; b < 3; ++b)
        for (int f = 0; f < 3; ++f) d->st[b][f] = (float *)take(L.field);
    d->rx = (float *)take(L.field);
    d->ry = (float *)take(L.field);
    for (int f = 0; f < 3; ++f) d->S[f] = (float *)take(L.field);
    for (int s = 0; s < 3; ++s)
        for (int f = 0; f < 5; ++f) d->hist[s][f] = (float *)take(L.field);
    d->D = (float *)take(L.corners);
    d->Dnew = (float *)take(L.corners);
    d->redx = (float4 *)take(L.redx);
    d->redy = (float4 *)take(L.redy);
    d->solx = (float *)take(L.solx);
    d->soly = (float *)take(L.soly);
    d->lux = (float *)take(L.lux);
    d->luy = (float *)take(L.luy);
    d->lu_valid = false;
    d->ghost[0] = (float *)take(L.ghost);
    d->ghost[1] = (float *)take(L.ghost);
    for (int s = 0; s < 4; ++s) d->tab[s] = (double *)take(L.tabs);
    char *misc = take(L.misc);
    d->health = (int *)misc;
    d->scal = (double *)(misc + 64);
    d->nvar = L.nvar;
    d->vsa = (StencilArgs *)take(L.vtab);
    d->vso = (SolveArgs *)(d->vsa + L.nvar);
    d->vdirty = true;
    d->sy = SY;
    d->pnt = PCR_NT;
    d->solver = WS_SOLVE_PCR;
    d->fstride = L.field;
    for (int s = 0; s < 4; ++s) { d->side_type[s] = WS_BC_SOLID; d->side_width[s] = 2; d->side_expo[s] = 1.f; }
    hipStream_t st = (hipStream_t)stream;
    // the whole layout starts at zero (a reused workspace keeps what its last
    // domain left there)
    hipError_t e = hipMemsetAsync(d->base, 0, L.total, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_corners_from_z, dim3((g->nx + 1 + 255) / 256, g->ny + 1), dim3(256), 0, st,
                           z_corners_dev, d->D, g->nx, g->ny, d->zpitch, (float)g->still_water);
        Dom m = make_dom(d);
        hipLaunchKernelGGL(k_rest_state, cells_grid(g->nx, g->ny), dim3(256), 0, st, m, d->st[0][0],
                           d->st[0][1], d->st[0][2]);
        hipLaunchKernelGGL(k_check_dd, cells_grid(g->nx, g->ny), dim3(256), 0, st, m, d->health);
        e = hipGetLastError();
    }
    int flag = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, d->health, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess && flag) e = hipMemsetAsync(d->health, 0, sizeof(int), st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(WS_EHIP, "%s: %s", who, hipGetErrorString(e));
    if (flag) return fail(WS_ENOTDD, "%s: bathymetry too steep for the grid (eq. 23 not diagonally dominant)", who);
    d->cur = 0;
    d->step = 0;
    d->t = 0.0;
    return WS_OK;
}

extern "C" ws_status ws_domain_init(const ws_grid *g, const float *z_corners_dev, void *workspace_dev,
                                    size_t workspace_bytes, void *stream, ws_domain **out) {
    if (!out) return fail(WS_EINVAL, "ws_domain_init: out is NULL");
    *out = nullptr;
    ws_status s = init_checks(g, z_corners_dev, workspace_dev, workspace_bytes, "ws_domain_init");
    if (s != WS_OK) return s;
    ws_domain *d = new (std::nothrow) ws_domain();
    if (!d) return fail(WS_ENOMEM, "ws_domain_init: host allocation failed");
    s = domain_setup(d, g, z_corners_dev, workspace_dev, workspace_bytes, stream, "ws_domain_init");
    if (s != WS_OK) {
        delete d;
        return s;
    }
    *out = d;
    return WS_OK;
}

// ---- A domain in the library's own device array, for callers that cannot
// allocate device memory.  `scratch` is one array per GPU (the code object
// holds it on every device it is loaded on until the process ends).  In host
// code its name is not a device address: the address is looked up once per
// device with hipGetSymbolAddress, with that device current, and only that
// pointer is used.  The handle lives in static storage too, so creating such
// a domain allocates nothing, on the device or on the host.  One such domain
// per device at a time.
static constexpr int STATIC_MAXDEV = 64;
static __device__ __align__(256) unsigned char scratch[WS_STATIC_WORKSPACE_BYTES];
static void *g_scratch_ptr[STATIC_MAXDEV];     // device address of `scratch`, per device
static bool g_scratch_held[STATIC_MAXDEV];     // a live domain uses that device's array
alignas(ws_domain) static unsigned char g_static_dom[STATIC_MAXDEV][sizeof(ws_domain)];
static std::mutex g_scratch_mu;

extern "C" ws_status ws_domain_init_static(const ws_grid *g, const float *z_corners_dev, void *stream,
                                           ws_domain **out) {
    static const char *who = "ws_domain_init_static";
    if (!out) return fail(WS_EINVAL, "%s: out is NULL", who);
    *out = nullptr;
    if (!grid_ok(g)) return fail(WS_EINVAL, "%s: invalid grid parameters", who);
    const size_t need = layout(g).total;
    if (need > WS_STATIC_WORKSPACE_BYTES)
        return fail(WS_ENOMEM, "%s: the grid needs %zu bytes of workspace, the static array holds %zu",
                    who, need, (size_t)WS_STATIC_WORKSPACE_BYTES);
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= STATIC_MAXDEV) return fail(WS_EINVAL, "%s: device %d out of range", who, dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_held[dev])
        return fail(WS_EBUSY, "%s: the static workspace of device %d is held by a live domain", who, dev);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(WS_EHIP, "%s: hipGetSymbolAddress: %s", who, hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    ws_status s = init_checks(g, z_corners_dev, g_scratch_ptr[dev], WS_STATIC_WORKSPACE_BYTES, who);
    if (s != WS_OK) return s;
    ws_domain *d = new (g_static_dom[dev]) ws_domain();
    s = domain_setup(d, g, z_corners_dev, g_scratch_ptr[dev], WS_STATIC_WORKSPACE_BYTES, stream, who);
    if (s != WS_OK) {
        d->~ws_domain();
        return s;
    }
    d->static_dev = dev;
    g_scratch_held[dev] = true;
    *out = d;
    return WS_OK;
}

static void prof_clear(ws_domain *d) {
    for (auto &e : d->prof) {
        (void)hipEventDestroy(e.second.first);
        (void)hipEventDestroy(e.second.second);
    }
    d->prof.clear();
}

extern "C" ws_status ws_domain_destroy(ws_domain *d) {
    if (d && d->batch) return fail(WS_EBUSY, "ws_domain_destroy: detach the domain from its batch first");
    if (!d) return WS_OK;
    prof_clear(d);
    if (d->static_dev >= 0) {  // a domain in the static array: release the array
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        const int dev = d->static_dev;
        d->~ws_domain();
        g_scratch_held[dev] = false;
        return WS_OK;
    }
    delete d;
    return WS_OK;
}

extern "C" ws_status ws_profile_enable(ws_domain *d, int32_t on) {
    if (!d) return fail(WS_EINVAL, "ws_profile_enable: NULL domain");
    d->prof_on = on != 0;
    return WS_OK;
}

extern "C" ws_status ws_profile_collect(ws_domain *d, void *stream, double *total_ms, int64_t *launches,
                                        int32_t n) {
    if (!d || n < 0 || (n > 0 && (!total_ms || !launches))) return fail(WS_EINVAL, "ws_profile_collect: bad argument");
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    for (auto &e : d->prof) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e.second.first, e.second.second));
        if (e.first < n) {
            total_ms[e.first] += ms;
            launches[e.first] += 1;
        }
    }
    prof_clear(d);
    return WS_OK;
}

// Event pair around one launch when profiling is on.
struct ProfScope {
    ws_domain *d;
    hipStream_t st;
    int cls;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(ws_domain *d_, hipStream_t s, int c) : d(d_), st(s), cls(c) {
        if (!d->prof_on) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) { a = b = nullptr; return; }
        (void)hipEventRecord(a, st);
    }
    ~ProfScope() {
        if (!a) return;
        (void)hipEventRecord(b, st);
        d->prof.push_back({cls, {a, b}});
    }
};

// Damping exponent of a sponge side: 1 for the layer of eq. 30, 0 for a
// wall; for a partially reflective layer, a long wave crossing it and coming
// back keeps the share exp(-4 s L ln 2 / (c dt)) of its amplitude.
static float sponge_expo(const ws_domain *d, int side) {
    const double R = d->side_R[side], dside = d->side_depth[side];
    if (R == 1.0) return 0.f;  // no damping: a solid wall
    if (!(R > 0.0) || !(dside > 0.0)) return 1.f;
    const double L = d->side_width[side] * (side < 2 ? d->g.dx : d->g.dy);
    const double e = -std::log(R) * std::sqrt(d->g.g * dside) * d->g.dt / (4.0 * L * std::log(2.0));
    return (float)(e < 1.0 ? e : 1.0);
}

extern "C" ws_status ws_set_boundary(ws_domain *d, int32_t side, const ws_boundary *b) {
    if (!d || !b || side < 0 || side > 3) return fail(WS_EINVAL, "ws_set_boundary: bad argument");
    if (busy_check(d, "ws_set_boundary") != WS_OK) return WS_EBUSY;
    if (b->type < 0 || b->type > 2) return fail(WS_EINVAL, "ws_set_boundary: bad type %d", b->type);
    const int nc = b->type == WS_BC_WAVES ? b->n_comp : 0;
    if (nc < 0 || nc > MAXC) return fail(WS_EINVAL, "ws_set_boundary: n_comp %d out of range", b->n_comp);
    if (b->type == WS_BC_SPONGE && b->width_cells < 1) return fail(WS_EINVAL, "ws_set_boundary: sponge width < 1");
    if (b->type == WS_BC_SPONGE && !(b->sponge_reflect >= 0.0 && b->sponge_reflect <= 1.0))
        return fail(WS_EINVAL, "ws_set_boundary: sponge_reflect must lie in [0, 1]");
    if (nc > 0 && (!b->amp || !b->period || !b->theta_rad)) return fail(WS_EINVAL, "ws_set_boundary: NULL component array");
    d->side_type[side] = b->type;
    d->side_width[side] = b->width_cells;
    d->side_ncomp[side] = 0;
    d->side_expo[side] = 1.f;
    const double R = b->type == WS_BC_SPONGE ? b->sponge_reflect : 0.0;
    double dref = b->ref_depth, dside = 0.0;
    if ((nc > 0 && !(dref > 0.0)) || (R > 0.0 && R < 1.0)) {
        Dom m = make_dom(d);
        hipLaunchKernelGGL(k_side_depth, dim3(1), dim3(256), 0, 0, m, side, d->scal);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpy(&dside, d->scal, sizeof(double), hipMemcpyDeviceToHost));
        if (!(dref > 0.0)) dref = dside;
    }
    d->side_R[side] = R;
    d->side_depth[side] = dside;
    d->side_expo[side] = sponge_expo(d, side);
    if (nc > 0 && !(dref > 0.0)) return fail(WS_EINVAL, "ws_set_boundary: no positive depth along the side");
    std::vector<double> tab((size_t)MAXC * TABW, 0.0);
    const double g = d->g.g;
    for (int m = 0; m < nc; ++m) {
        if (!(b->period[m] > 0.0)) return fail(WS_EINVAL, "ws_set_boundary: period must be > 0");
        const double om = 2.0 * M_PI / b->period[m];
        // Eckart's approximation of the linear dispersion relation (eq. 29)
        const double k = om * om / g * std::sqrt(1.0 / std::tanh(om * om * dref / g));
        const double c = om / k, cth = std::cos(b->theta_rad[m]), sth = std::sin(b->theta_rad[m]);
        double *r = &tab[(size_t)m * TABW];
        r[0] = b->amp[m];
        r[1] = om;
        r[2] = k * cth;
        r[3] = k * sth;
        r[4] = c * cth;
        r[5] = c * sth;
        r[6] = b->phase ? b->phase[m] : 0.0;
    }
    HIPCHK(hipMemcpy(d->tab[side], tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
    d->side_ncomp[side] = nc;
    d->lu_valid = false;  // boundary rows of the reduced systems change
    batch_touch(d);
    return WS_OK;
}

extern "C" ws_status ws_update_grid(ws_domain *d, const ws_grid *g, void *stream) {
    if (!d || !g) return fail(WS_EINVAL, "ws_update_grid: bad argument");
    if (busy_check(d, "ws_update_grid") != WS_OK) return WS_EBUSY;
    const ws_grid &o = d->g;
    if (g->nx != o.nx || g->ny != o.ny || g->dx != o.dx || g->dy != o.dy || g->n_corr != o.n_corr ||
        g->still_water != o.still_water)
        return fail(WS_EINVAL, "ws_update_grid: nx, ny, dx, dy, n_corr and still_water are fixed at init");
    if (!grid_ok(g) || !(g->Bcoef >= 0.0) || !(g->friction_coef >= 0.0))
        return fail(WS_EINVAL, "ws_update_grid: parameter out of range");
    const bool systems = g->model != o.model || g->Bcoef != o.Bcoef;  // eq. 23 coefficients change
    if (systems) {
        hipStream_t st = (hipStream_t)stream;
        Dom m = make_dom(d);
        m.model = g->model;
        m.Bd = (float)g->Bcoef;
        int flag = 0;
        hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, st, reinterpret_cast<unsigned *>(d->scal), 1);
        hipLaunchKernelGGL(k_check_dd, cells_grid(d->g.nx, d->g.ny), dim3(256), 0, st, m, (int *)d->scal);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(&flag, d->scal, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (flag) return fail(WS_ENOTDD, "ws_update_grid: eq. 23 would lose diagonal dominance");
    }
    const bool restart = g->dt != o.dt;
    d->g = *g;
    if (restart) {
        // the multistep history assumes one time step: restart it (the next
        // two steps are Euler steps, as after a hot start); the partially
        // reflective sponges scale with the time step
        d->step = 0;
        for (int q = 0; q < 4; ++q)
            if (d->side_type[q] == WS_BC_SPONGE) d->side_expo[q] = sponge_expo(d, q);
    }
    if (systems) d->lu_valid = false;
    batch_touch(d);
    return WS_OK;
}

// ------------------------------------------------------- snapshot / restore
// Snapshot layout: a 256-byte header, then the current state (eta, P, Q), the
// three history slots (E, F, G, F*, G* each) and the corner depth, each as
// the domain stores it (padded rows).
struct SnapHeader {
    unsigned long long magic;
    int nx, ny, pitch, zpitch;
    long long step;
    double t, dt;
    int n_corr, model;
    unsigned long long field_bytes, corner_bytes, total;
};
static_assert(sizeof(SnapHeader) <= 256, "the snapshot header fills the first 256 bytes");
static const unsigned long long SNAP_MAGIC = 0x3230504e53535757ull;  // "WWSSNP02"

extern "C" size_t ws_snapshot_bytes_grid(const ws_grid *g) {
    if (!grid_ok(g)) return 0;
    const Layout L = layout(g);
    return 256 + 18 * sizeof(float) * (size_t)L.nyp * L.pitch + sizeof(float) * (size_t)(g->ny + 1) * L.zpitch;
}

static size_t snap_field_bytes(const ws_domain *d) { return sizeof(float) * (size_t)d->nyp * d->pitch; }
static size_t snap_corner_bytes(const ws_domain *d) { return sizeof(float) * (size_t)(d->g.ny + 1) * d->zpitch; }

extern "C" size_t ws_snapshot_bytes(const ws_domain *d) {
    if (!d) return 0;
    return 256 + 18 * snap_field_bytes(d) + snap_corner_bytes(d);
}

__global__ void k_snap_header(SnapHeader h, SnapHeader *dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = h;
}

extern "C" ws_status ws_snapshot(ws_domain *d, void *dst_dev, size_t bytes, void *stream) {
    if (!d || !dst_dev) return fail(WS_EINVAL, "ws_snapshot: bad argument");
    if (busy_check(d, "ws_snapshot") != WS_OK) return WS_EBUSY;
    if (((uintptr_t)dst_dev & 255) != 0) return fail(WS_EINVAL, "ws_snapshot: buffer not 256-byte aligned");
    const size_t need = ws_snapshot_bytes(d), fb = snap_field_bytes(d), cb = snap_corner_bytes(d);
    if (bytes < need) return fail(WS_ENOMEM, "ws_snapshot: buffer %zu < %zu bytes", bytes, need);
    hipStream_t st = (hipStream_t)stream;
    SnapHeader h;
    std::memset(&h, 0, sizeof h);
    h.magic = SNAP_MAGIC;
    h.nx = d->g.nx; h.ny = d->g.ny; h.pitch = d->pitch; h.zpitch = d->zpitch;
    h.step = d->step; h.t = d->t; h.dt = d->g.dt;
    h.n_corr = d->g.n_corr; h.model = d->g.model;
    h.field_bytes = fb; h.corner_bytes = cb; h.total = need;
    char *p = (char *)dst_dev;
    hipLaunchKernelGGL(k_snap_header, dim3(1), dim3(64), 0, st, h, (SnapHeader *)p);
    p += 256;
    for (int f = 0; f < 3; ++f, p += fb) HIPCHK(hipMemcpyAsync(p, d->st[d->cur][f], fb, hipMemcpyDeviceToDevice, st));
    for (int sl = 0; sl < 3; ++sl)
        for (int f = 0; f < 5; ++f, p += fb) HIPCHK(hipMemcpyAsync(p, d->hist[sl][f], fb, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(p, d->D, cb, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipGetLastError());
    return WS_OK;
}

extern "C" ws_status ws_restore(ws_domain *d, const void *src_dev, size_t bytes, void *stream) {
    if (!d || !src_dev) return fail(WS_EINVAL, "ws_restore: bad argument");
    if (busy_check(d, "ws_restore") != WS_OK) return WS_EBUSY;
    const size_t need = ws_snapshot_bytes(d), fb = snap_field_bytes(d), cb = snap_corner_bytes(d);
    if (bytes < need) return fail(WS_EINVAL, "ws_restore: buffer %zu < %zu bytes", bytes, need);
    hipStream_t st = (hipStream_t)stream;
    SnapHeader h;
    HIPCHK(hipMemcpyAsync(&h, src_dev, sizeof h, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (h.magic != SNAP_MAGIC || h.nx != d->g.nx || h.ny != d->g.ny || h.pitch != d->pitch ||
        h.zpitch != d->zpitch || h.total != need || h.n_corr != d->g.n_corr || h.model != d->g.model)
        return fail(WS_EINVAL, "ws_restore: snapshot does not match this domain's grid");
    const char *p = (const char *)src_dev + 256;
    for (int f = 0; f < 3; ++f, p += fb) HIPCHK(hipMemcpyAsync(d->st[0][f], p, fb, hipMemcpyDeviceToDevice, st));
    for (int sl = 0; sl < 3; ++sl)
        for (int f = 0; f < 5; ++f, p += fb) HIPCHK(hipMemcpyAsync(d->hist[sl][f], p, fb, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(d->D, p, cb, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemsetAsync(d->health, 0, sizeof(int), st));
    d->cur = 0;
    // history levels taken at another time step are not spaced by this one:
    // the multistep history restarts (two Euler steps), as after a change of dt
    d->step = h.dt == d->g.dt ? h.step : 0;
    d->t = h.t;
    d->lu_valid = false;  // bathymetry restored
    batch_touch(d);
    return WS_OK;
}

extern "C" ws_status ws_set_state(ws_domain *d, const float *w, const float *P, const float *Q,
                                  int32_t pitch, double t, void *stream) {
    if (!d || !w || !P || !Q || pitch < d->g.nx) return fail(WS_EINVAL, "ws_set_state: bad argument");
    if (busy_check(d, "ws_set_state") != WS_OK) return WS_EBUSY;
    Dom m = make_dom(d);
    hipLaunchKernelGGL(k_set_state, cells_grid(d->g.nx, d->g.ny), dim3(256), 0, (hipStream_t)stream, m, w, P,
                       Q, pitch, (float)d->g.still_water, d->st[d->cur][0], d->st[d->cur][1], d->st[d->cur][2]);
    HIPCHK(hipGetLastError());
    d->t = t;
    d->step = 0;
    batch_touch(d);
    return WS_OK;
}

extern "C" ws_status ws_read(ws_domain *d, int32_t what, float *first, float *P, float *Q,
                             int32_t pitch, void *stream) {
    if (!d || pitch < d->g.nx || (what != WS_READ_W && what != WS_READ_H)) return fail(WS_EINVAL, "ws_read: bad argument");
    if (busy_check(d, "ws_read") != WS_OK) return WS_EBUSY;
    Dom m = make_dom(d);
    hipLaunchKernelGGL(k_read, cells_grid(d->g.nx, d->g.ny), dim3(256), 0, (hipStream_t)stream, m,
                       d->st[d->cur][0], d->st[d->cur][1], d->st[d->cur][2], what, (float)d->g.still_water,
                       first, P, Q, pitch);
    HIPCHK(hipGetLastError());
    return WS_OK;
}

extern "C" ws_status ws_read_gauges(ws_domain *d, int32_t n, const int32_t *ij_dev, float *out_dev,
                                    void *stream) {
    if (!d || n < 0 || (n > 0 && (!ij_dev || !out_dev))) return fail(WS_EINVAL, "ws_read_gauges: bad argument");
    if (busy_check(d, "ws_read_gauges") != WS_OK) return WS_EBUSY;
    if (n == 0) return WS_OK;
    Dom m = make_dom(d);
    hipLaunchKernelGGL(k_gauges, dim3((n + 63) / 64), dim3(64), 0, (hipStream_t)stream, m, d->st[d->cur][0],
                       d->st[d->cur][1], d->st[d->cur][2], (float)d->g.still_water, ij_dev, n, out_dev);
    HIPCHK(hipGetLastError());
    return WS_OK;
}

extern "C" ws_status ws_add_solitary(ws_domain *d, double H, double theta, double x0, double y0,
                                     void *stream) {
    if (!d) return fail(WS_EINVAL, "ws_add_solitary: NULL domain");
    if (busy_check(d, "ws_add_solitary") != WS_OK) return WS_EBUSY;
    hipStream_t st = (hipStream_t)stream;
    // still water depth of the bilinear bottom at (x0, y0)
    double fx = x0 / d->g.dx, fy = y0 / d->g.dy;
    int ci = (int)std::floor(fx), cj = (int)std::floor(fy);
    ci = ci < 0 ? 0 : (ci > d->g.nx - 1 ? d->g.nx - 1 : ci);
    cj = cj < 0 ? 0 : (cj > d->g.ny - 1 ? d->g.ny - 1 : cj);
    float c[4];
    HIPCHK(hipStreamSynchronize(st));
    for (int k = 0; k < 4; ++k)
        HIPCHK(hipMemcpy(&c[k], d->D + (size_t)(cj + k / 2) * d->zpitch + ci + k % 2, sizeof(float),
                         hipMemcpyDeviceToHost));
    double ax = fx - ci, ay = fy - cj;
    double dep = (1 - ax) * (1 - ay) * c[0] + ax * (1 - ay) * c[1] + (1 - ax) * ay * c[2] + ax * ay * c[3];
    if (!(dep > 0.0) || !(H + dep > 0.0)) return fail(WS_EINVAL, "ws_add_solitary: no positive depth at the crest");
    const double ks = std::sqrt(3.0 * std::fabs(H) / (4.0 * dep * dep * dep));  // eq. 35
    const double cs = std::sqrt(d->g.g * (H + dep));                            // eq. 36
    Dom m = make_dom(d);
    hipLaunchKernelGGL(k_solitary, cells_grid(d->g.nx, d->g.ny), dim3(256), 0, st, m, d->st[d->cur][0],
                       d->st[d->cur][1], d->st[d->cur][2], H, ks, cs, std::cos(theta), std::sin(theta), x0, y0);
    HIPCHK(hipGetLastError());
    return WS_OK;
}

extern "C" ws_status ws_apply_edit(ws_domain *d, int32_t kind, double x0, double y0, double amp,
                                   double sigma, void *stream) {
    if (!d || !(sigma > 0.0)) return fail(WS_EINVAL, "ws_apply_edit: bad argument");
    if (busy_check(d, "ws_apply_edit") != WS_OK) return WS_EBUSY;
    hipStream_t st = (hipStream_t)stream;
    Dom m = make_dom(d);
    float *e = d->st[d->cur][0], *p = d->st[d->cur][1], *q = d->st[d->cur][2];
    if (kind == WS_EDIT_ADD_WATER) {
        hipLaunchKernelGGL(k_edit_water, cells_grid(d->g.nx, d->g.ny), dim3(256), 0, st, m, e, p, q, x0, y0,
                           amp, sigma);
        HIPCHK(hipGetLastError());
        return WS_OK;
    }
    if (kind != WS_EDIT_RAISE_TERRAIN) return fail(WS_EINVAL, "ws_apply_edit: bad kind %d", kind);
    hipLaunchKernelGGL(k_edit_terrain, cells_grid(d->g.nx + 1, d->g.ny + 1), dim3(256), 0, st, m, d->D,
                       d->Dnew, x0, y0, amp, sigma);
    Dom mn = m;
    mn.D = d->Dnew;
    HIPCHK(hipMemsetAsync(d->scal, 0, sizeof(int), st));
    hipLaunchKernelGGL(k_check_dd, cells_grid(d->g.nx, d->g.ny), dim3(256), 0, st, mn, (int *)d->scal);
    HIPCHK(hipGetLastError());
    int flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, d->scal, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (flag) return fail(WS_ENOTDD, "ws_apply_edit: terrain edit rejected (eq. 23 would lose diagonal dominance)");
    std::swap(d->D, d->Dnew);
    d->lu_valid = false;
    batch_touch(d);
    m = make_dom(d);
    hipLaunchKernelGGL(k_edit_velocity, cells_grid(d->g.nx, d->g.ny), dim3(256), 0, st, m, d->Dnew, e, p, q);
    hipLaunchKernelGGL(k_shore_fix, cells_grid(d->g.nx, d->g.ny), dim3(256), 0, st, m, e, p, q);
    HIPCHK(hipGetLastError());
    return WS_OK;
}

// Stencil workgroup grid: SWG side-by-side strips of sy rows per workgroup,
// or (solo) one strip per workgroup.
static dim3 strips_for(const ws_domain *d, int sy, bool solo = false) {
    const int ns = (d->g.nx + SO - 1) / SO;
    return dim3(solo ? ns : (ns + SWG - 1) / SWG, (d->g.ny + sy - 1) / sy);
}

#define SY_SWITCH(K, sy, LAUNCH)                        \
    do {                                                \
        if (sy == 8) LAUNCH(K<8>);                      \
        else if (sy == 16) LAUNCH(K<16>);               \
        else if (sy == 24) LAUNCH(K<24>);               \
        else if (sy == 48) LAUNCH(K<48>);               \
        else if (sy == 64) LAUNCH(K<64>);               \
        else LAUNCH(K<32>);                             \
    } while (0)

// The workgroup shape follows the kernel: the corrector runs one-wave
// workgroups, the predictors SWG strips a workgroup.
static void launch_stencil(const ws_domain *d, int sy, hipStream_t st, const StencilArgs &sa) {
    const bool solo = sa.kind == 2;
    const dim3 grid = strips_for(d, sy, solo);
    const dim3 g1(grid.x * grid.y);  // 1-D grid in XCD-aware tile order
    const int gx = (int)grid.x;
#define L3(KERN) hipLaunchKernelGGL(KERN, g1, dim3(solo ? 64 : 64 * SWG), 0, st, sa, gx)
    if (sa.kind == 2) SY_SWITCH(k_stencil_c, sy, L3);
    else if (sa.kind == 1) SY_SWITCH(k_stencil_p, sy, L3);
    else SY_SWITCH(k_stencil_e, sy, L3);
#undef L3
}
// Equations per thread for systems of up to nred unknowns: a power of two.
static int pcr_epl(int pnt, int nred) {
    int e = 1;
    while (e * pnt < nred) e *= 2;
    return e;
}

// Launches by (threads per system, equations per thread); `Go` is called
// with the kernel's template arguments as a tag.
template <int PNT, int EPL> struct PcrShape {
    static constexpr int threads = PNT, epl = EPL;
};
template <class Go> static void pcr_dispatch(int pnt, int epl, Go go) {
    if (pnt == 64) {
        if (epl <= 1) go(PcrShape<64, 1>());
        else if (epl <= 2) go(PcrShape<64, 2>());
        else if (epl <= 4) go(PcrShape<64, 4>());
        else if (epl <= 8) go(PcrShape<64, 8>());
        else if (epl <= 16) go(PcrShape<64, 16>());
        else go(PcrShape<64, 32>());
    } else if (pnt == 256) {
        if (epl <= 1) go(PcrShape<256, 1>());
        else if (epl <= 2) go(PcrShape<256, 2>());
        else if (epl <= 4) go(PcrShape<256, 4>());
        else go(PcrShape<256, 8>());
    } else {
        if (epl <= 1) go(PcrShape<128, 1>());
        else if (epl <= 2) go(PcrShape<128, 2>());
        else if (epl <= 4) go(PcrShape<128, 4>());
        else if (epl <= 8) go(PcrShape<128, 8>());
        else go(PcrShape<128, 16>());
    }
}

static void launch_pcr(int pnt, int nred, int nsys, hipStream_t st, const SolveArgs &so) {
    const size_t shm = sizeof(float4) * nred;
    pcr_dispatch(pnt, pcr_epl(pnt, nred), [&](auto shape) {
        using S = decltype(shape);
        hipLaunchKernelGGL((k_pcr<S::threads, S::epl>), dim3(nsys), dim3(S::threads), shm, st, so);
    });
}

// The wave form of PCR (one wave per system, lane shuffles): equations per
// lane the next power of two of nred / 64; systems of up to 512 unknowns.
static bool pcrw_fits(int nred) { return nred <= 64 * PCRW_EPL_MAX; }
static void launch_pcrw(int nred, int nsys, hipStream_t st, const SolveArgs &so) {
    if (nred <= 64) hipLaunchKernelGGL(k_pcrw<1>, dim3(nsys), dim3(64), 0, st, so);
    else if (nred <= 128) hipLaunchKernelGGL(k_pcrw<2>, dim3(nsys), dim3(64), 0, st, so);
    else if (nred <= 256) hipLaunchKernelGGL(k_pcrw<4>, dim3(nsys), dim3(64), 0, st, so);
    else hipLaunchKernelGGL(k_pcrw<8>, dim3(nsys), dim3(64), 0, st, so);
}

static void launch_pcrw_batch(int nred, dim3 pg, hipStream_t st, const BatchDesc *desc, const BatchState *state,
                              const int *pre, int n, int p) {
    if (nred <= 64) hipLaunchKernelGGL(kb_pcrw<1>, pg, dim3(64), 0, st, desc, state, pre, n, p);
    else if (nred <= 128) hipLaunchKernelGGL(kb_pcrw<2>, pg, dim3(64), 0, st, desc, state, pre, n, p);
    else if (nred <= 256) hipLaunchKernelGGL(kb_pcrw<4>, pg, dim3(64), 0, st, desc, state, pre, n, p);
    else hipLaunchKernelGGL(kb_pcrw<8>, pg, dim3(64), 0, st, desc, state, pre, n, p);
}

// One predictor or corrector pass: stencil, then the partitioned solves.
// Arguments of pass p of a step.  cur: state buffer of the step's state;
// sm: step index mod 3 (history slots); euler: one of the two start-up steps.
static void pass_args(const ws_domain *d, const Dom &m, bool euler, int cur, int sm, int p, StencilArgs &sa,
                      SolveArgs &so) {
    const ws_grid &g = d->g;
    const int K = euler ? 0 : g.n_corr;
    const int n0 = (sm + 2) % 3, n1 = (sm + 1) % 3, n2 = sm;
    const int a = cur, b = (a + 1) % 3, c = (a + 2) % 3;
    const int in = p == 0 ? a : ((p & 1) ? b : c);
    const int out = p == 0 ? b : ((p & 1) ? c : b);
    std::memset(&sa, 0, sizeof sa);
    sa.d = m;
    sa.d.gh = d->ghost[p == 0 ? 0 : 1];
    sa.in = d->st[in][0];
    sa.eout = d->st[out][0];
    sa.rxy = d->rx;
    sa.h0 = d->hist[n0][0];
    sa.h1 = d->hist[n1][0];
    sa.h2 = d->hist[n2][0];
    sa.S = d->S[0];
    sa.fstride = (unsigned)d->fstride;
    {
        const double rx = 1.0 / g.dx, ry = 1.0 / g.dy;
        sa.hx = (float)(0.5 * rx);
        sa.hy = (float)(0.5 * ry);
        sa.sxx = (float)(rx * rx);
        sa.syy = (float)(ry * ry);
        sa.cxy = (float)(0.25 * rx * ry);
        sa.cxxx = (float)(0.5 * rx * rx * rx);
        sa.cyyy = (float)(0.5 * ry * ry * ry);
        sa.cxyy = (float)(0.5 * rx * ry * ry);
        sa.cxxy = (float)(0.5 * rx * rx * ry);
        sa.gx = (float)(g.g * rx);
        sa.gy = (float)(g.g * ry);
        sa.Bg = (float)(g.Bcoef * g.g);
    }
    sa.dt = (float)g.dt;
    sa.x0 = sa.x1 = sa.x2 = 0.f;
    if (g.fstar_extrap == 2) { sa.x0 = 2.f; sa.x1 = -3.f; sa.x2 = 1.f; }
    else if (g.fstar_extrap == 1) { sa.x0 = 1.f; sa.x1 = -1.f; }
    sa.kind = p == 0 ? (euler ? 0 : 1) : 2;
    sa.write_S = (p == 0 && !euler && K > 0) ? 1 : 0;
    std::memset(&so, 0, sizeof so);
    so.d = sa.d;
    so.rx = d->rx;
    so.ry = d->ry;
    so.redx = d->redx;
    so.redy = d->redy;
    so.solx = d->solx;
    so.soly = d->soly;
    so.eta = d->st[out][0];
    so.pout = d->st[out][1];
    so.qout = d->st[out][2];
    so.pbase = d->st[a][1];
    so.qbase = d->st[a][2];
    so.gh0 = d->ghost[0];
    so.gh1 = d->ghost[1];
    so.health = d->health;
    so.lux = d->lux;
    so.luy = d->luy;
    so.layout = (d->solver == WS_SOLVE_LU || d->solver == WS_SOLVE_LU2) ? 1 : 0;
    so.sponge = p == K ? 1 : 0;
    so.nlsw = g.model == WS_NLSW ? 1 : 0;
}

static bool has_makers(const ws_domain *d) {
    for (int q = 0; q < 4; ++q)
        if (d->side_type[q] == WS_BC_WAVES) return true;
    return false;
}

static int solve_waves(const ws_domain *d) { return (d->g.ny + 63) / 64 + (d->g.nx + 63) / 64; }
static int solve2_waves(int nx, int ny) { return (2 * ny + 63) / 64 + (2 * nx + 63) / 64; }
// Waves per workgroup of the one-ended factored solve's workgroup form (LUR
// unknowns a wave), or 0 where the longest reduced system is too long for it
// and the lane-per-system sweep runs instead.
static int luw_waves(int nred) { return nred <= LUR * LUW_MAX ? (nred + LUR - 1) / LUR : 0; }
static int luw_groups(int nx, int ny) { return (ny + LUS - 1) / LUS + (nx + LUS - 1) / LUS; }
static int nred_of(const ws_domain *d) { return d->nu > d->nv ? d->nu : d->nv; }
static bool factored(int solver) { return solver == WS_SOLVE_LU || solver == WS_SOLVE_LU2; }

// Factors of the reduced systems for the factored solve, when stale: a
// coefficient-mode reduction (contiguous equations; its right-hand sides and
// eliminated values are scratch) and one factorization sweep per system.
static ws_status ensure_factors(ws_domain *d, hipStream_t st) {
    if (!factored(d->solver) || (d->lu_valid && d->lu_kind == d->solver)) return WS_OK;
    StencilArgs sa;
    SolveArgs so;
    pass_args(d, make_dom(d), false, d->cur, 0, 0, sa, so);
    so.layout = 0;
    hipLaunchKernelGGL(k_reduce, tiles(d), dim3(NT), 0, st, so);
    if (d->solver == WS_SOLVE_LU2)
        hipLaunchKernelGGL(k_lu2_factor, dim3(solve_waves(d)), dim3(64), 0, st, so, d->lux, d->luy);
    else
        hipLaunchKernelGGL(k_lu_factor, dim3(solve_waves(d)), dim3(64), 0, st, so, d->lux, d->luy);
    HIPCHK(hipGetLastError());
    d->lu_valid = true;
    d->lu_kind = d->solver;
    return WS_OK;
}

// The reduced row and column systems, by the domain's strategy.
static void launch_reduced(const ws_domain *d, hipStream_t st, const SolveArgs &so) {
    if (d->solver == WS_SOLVE_LU2) {
        hipLaunchKernelGGL(k_lu2_solve, dim3(solve2_waves(d->g.nx, d->g.ny)), dim3(64), 0, st, so);
    } else if (d->solver == WS_SOLVE_LU) {
        const int G = luw_waves(nred_of(d));
        if (G)
            hipLaunchKernelGGL(k_luw_solve, dim3(luw_groups(d->g.nx, d->g.ny)), dim3(64 * G), 0, st, so);
        else
            hipLaunchKernelGGL(k_lu_solve, dim3(solve_waves(d)), dim3(64), 0, st, so);
    } else if (d->solver == WS_SOLVE_THOMAS) {
        const int waves = (d->g.ny + 63) / 64 + (d->g.nx + 63) / 64;
        hipLaunchKernelGGL(k_thomas, dim3(waves), dim3(64), 0, st, so);
    } else if (d->solver == WS_SOLVE_PCR_WAVE) {
        launch_pcrw(nred_of(d), d->g.ny + d->g.nx, st, so);
    } else {
        const int nred = d->nu > d->nv ? d->nu : d->nv;
        launch_pcr(d->pnt, nred, d->g.ny + d->g.nx, st, so);
    }
}

static ws_status run_pass(ws_domain *d, const StencilArgs &sa, const SolveArgs &so, hipStream_t st) {
    {
        ProfScope p(d, st, sa.kind == 2 ? WS_K_CORRECTOR : WS_K_PREDICTOR);
        const int rows = sa.kind == 2 && d->syc ? d->syc : d->sy;
        launch_stencil(d, rows, st, sa);
    }
    if (!so.nlsw) {  // NLSW: identity systems, nothing to solve
        {
            ProfScope p(d, st, WS_K_REDUCE);
            hipLaunchKernelGGL(k_reduce, tiles(d), dim3(NT), 0, st, so);
        }
        {
            ProfScope p(d, st, WS_K_SOLVE);
            launch_reduced(d, st, so);
        }
    }
    {
        ProfScope p(d, st, WS_K_EXPAND);
        hipLaunchKernelGGL(k_expand, tiles(d), dim3(NT), 0, st, so);
    }
    HIPCHK(hipGetLastError());
    return WS_OK;
}

extern "C" ws_status ws_advance(ws_domain *d, int64_t nsteps, void *stream) {
    if (!d || nsteps < 0) return fail(WS_EINVAL, "ws_advance: bad argument");
    if (d->batch) return fail(WS_EBUSY, "ws_advance: domain is attached to a batch (use ws_batch_advance)");
    hipStream_t st = (hipStream_t)stream;
    if (nsteps > 0) {
        ws_status r = ensure_factors(d, st);
        if (r != WS_OK) return r;
    }
    const Dom m = make_dom(d);
    const bool makers = has_makers(d);
    const bool conv = d->tol_w > 0.0;
    bool sponges = false;
    for (int q = 0; q < 4; ++q) sponges = sponges || d->side_type[q] == WS_BC_SPONGE;
    unsigned *dres = reinterpret_cast<unsigned *>(reinterpret_cast<char *>(d->health) + 128);
    for (int64_t n = 0; n < nsteps; ++n) {
        const int64_t s = d->step + 1;
        const bool euler = s <= 2;
        int K = euler ? 0 : d->g.n_corr;
        const double t0 = d->t, t1 = d->t + d->g.dt;
        if (makers) {
            const int n = 8 * d->gl * GHL;
            hipLaunchKernelGGL(k_ghosts, dim3((n + 255) / 256), dim3(256), 0, st, m, d->ghost[0], t0);
            hipLaunchKernelGGL(k_ghosts, dim3((n + 255) / 256), dim3(256), 0, st, m, d->ghost[1], t1);
        }
        StencilArgs sa;
        SolveArgs so;
        for (int p = 0; p <= K; ++p) {
            pass_args(d, m, euler, d->cur, (int)(s % 3), p, sa, so);
            if (conv) so.sponge = 0;  // applied once the count is known
            ws_status r = run_pass(d, sa, so, st);
            if (r != WS_OK) return r;
            if (conv && p >= 1) {
                // change against the previous iterate (the pass's input state)
                const int a = d->cur, b1 = (a + 1) % 3, c1 = (a + 2) % 3;
                const int in = (p & 1) ? b1 : c1, out = (p & 1) ? c1 : b1;
                hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, st, dres, 2);
                const int nb = std::min(1024, (d->g.nx * d->g.ny + 255) / 256);
                hipLaunchKernelGGL(k_residual, dim3(nb), dim3(256), 0, st, m, d->st[in][0], d->st[in][1],
                                   d->st[in][2], d->st[out][0], d->st[out][1], d->st[out][2], dres);
                unsigned h[2] = {0u, 0u};
                HIPCHK(hipMemcpyAsync(h, dres, sizeof h, hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
                float fw, fq;
                std::memcpy(&fw, &h[0], 4);
                std::memcpy(&fq, &h[1], 4);
                d->last_dw = fw;
                d->last_dpq = fq;
                if (fw <= d->tol_w && fq <= d->tol_pq) {
                    K = p;
                    break;
                }
            }
        }
        const int b = (d->cur + 1) % 3, c = (d->cur + 2) % 3;
        d->cur = K == 0 ? b : ((K & 1) ? c : b);
        if (conv) {
            if (sponges)
                hipLaunchKernelGGL(k_sponge, cells_grid(d->g.nx, d->g.ny), dim3(256), 0, st, m, d->st[d->cur][0],
                                   d->st[d->cur][1], d->st[d->cur][2]);
            d->last_corr = K;
            d->total_corr += K;
        }
        d->step = s;
        d->t = t1;
    }
    return WS_OK;
}

extern "C" ws_status ws_query(ws_domain *d, void *stream, int64_t *step, double *t, int32_t *health) {
    if (!d) return fail(WS_EINVAL, "ws_query: NULL domain");
    if (busy_check(d, "ws_query") != WS_OK) return WS_EBUSY;
    hipStream_t st = (hipStream_t)stream;
    int h = 0;
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(&h, d->health, sizeof(int), hipMemcpyDeviceToHost));
    if (step) *step = d->step;
    if (t) *t = d->t;
    if (health) *health = h;
    if (h) return fail(WS_ENONFINITE, "ws_query: non-finite state");
    return WS_OK;
}

extern "C" ws_status ws_set_corrector_tolerance(ws_domain *d, double tol_w, double tol_pq) {
    if (!d || tol_w != tol_w || tol_pq != tol_pq) return fail(WS_EINVAL, "ws_set_corrector_tolerance: bad argument");
    if (d->batch) return fail(WS_EBUSY, "ws_set_corrector_tolerance: domain is attached to a batch");
    d->tol_w = tol_w;
    d->tol_pq = tol_pq;
    d->last_corr = 0;
    d->total_corr = 0;
    d->last_dw = d->last_dpq = 0.0;
    return WS_OK;
}

extern "C" ws_status ws_corrector_stats(const ws_domain *d, int32_t *last, int64_t *total, double *dw, double *dpq) {
    if (!d) return fail(WS_EINVAL, "ws_corrector_stats: NULL domain");
    if (last) *last = d->last_corr;
    if (total) *total = d->total_corr;
    if (dw) *dw = d->last_dw;
    if (dpq) *dpq = d->last_dpq;
    return WS_OK;
}

// ------------------------------------------------------------------ batches
struct ws_batch {
    int max;
    BatchDesc *d_desc;
    BatchState *d_state;
    int *d_pre[5];                       // prefix tables: stencil, tile, pcr, ghost, corrector-stencil workgroups
    std::vector<ws_domain *> slots;      // attached domains by slot (nullptr = free)
    std::vector<int> order;              // slots in device table order
    std::vector<BatchState> h_state;     // host copy, device table order
    bool dirty = true;                   // tables must be rebuilt and uploaded
    bool stale = false;                  // device states ahead of the domains' host copies
    int maxK = 0, nred = 0, total[5] = {0, 0, 0, 0, 0};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t gstream = nullptr;
    hipStream_t last = nullptr;
    int sy = SY, pnt = PCR_NT, solver = WS_SOLVE_PCR;  // tuning shared by all domains of the batch
    int syc = 0;                                        // corrector-pass stencil rows (0: sy)
};

static size_t batch_layout(int max, size_t *o_state, size_t *o_pre) {
    size_t a = align256(sizeof(BatchDesc) * (size_t)max);
    size_t b = align256(sizeof(BatchState) * (size_t)max);
    size_t c = align256(sizeof(int) * (size_t)(max + 1));
    if (o_state) *o_state = a;
    if (o_pre) *o_pre = a + b;
    return a + b + 5 * c;
}

static void batch_touch(ws_domain *d) {
    if (!d) return;
    d->vdirty = true;
    if (d->batch) d->batch->dirty = true;
}

static void batch_drop_graph(ws_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->gstream = nullptr;
}

static BatchDesc make_desc(const ws_domain *d, int sy) {
    BatchDesc D;
    std::memset(&D, 0, sizeof D);
    D.d = make_dom(d);
    D.sa = d->vsa;
    D.so = d->vso;
    D.ghost[0] = d->ghost[0];
    D.ghost[1] = d->ghost[1];
    D.dt = d->g.dt;
    D.K = d->g.n_corr;
    const dim3 sg = strips_for(d, sy);
    D.sgx = (int)sg.x;
    D.sgy = (int)sg.y;
    D.sgxc = (int)strips_for(d, sy, true).x;
    D.tgx = d->nxp / TX;
    D.tgy = d->nyp / TY;
    D.nsys = d->g.ny + d->g.nx;
    D.makers = 0;
    for (int q = 0; q < 4; ++q) D.makers += d->side_type[q] == WS_BC_WAVES;
    D.health = d->health;
    return D;
}

// Pass argument tables of one domain (device), in the order of variant().
static ws_status write_vtab(ws_domain *d) {
    std::vector<StencilArgs> sa(d->nvar);
    std::vector<SolveArgs> so(d->nvar);
    const Dom m = make_dom(d);
    for (int key = 0; key < 9; ++key) {
        const int cur = key / 3, sm = key % 3;
        pass_args(d, m, true, cur, sm, 0, sa[key], so[key]);
        for (int p = 0; p <= d->g.n_corr; ++p) {
            const int v = 9 + key * (d->g.n_corr + 1) + p;
            pass_args(d, m, false, cur, sm, p, sa[v], so[v]);
        }
    }
    HIPCHK(hipMemcpy(d->vsa, sa.data(), sizeof(StencilArgs) * d->nvar, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(d->vso, so.data(), sizeof(SolveArgs) * d->nvar, hipMemcpyHostToDevice));
    d->vdirty = false;
    return WS_OK;
}

// Device states -> the domains' host copies.
static ws_status batch_pull(ws_batch *b, hipStream_t st) {
    if (!b->stale) return WS_OK;
    HIPCHK(hipStreamSynchronize(st));
    const int n = (int)b->order.size();
    if (n) HIPCHK(hipMemcpy(b->h_state.data(), b->d_state, sizeof(BatchState) * n, hipMemcpyDeviceToHost));
    for (int k = 0; k < n; ++k) {
        ws_domain *d = b->slots[b->order[k]];
        d->step = b->h_state[k].step;
        d->t = b->h_state[k].t;
        d->cur = b->h_state[k].cur;
        d->bhealth = b->h_state[k].health;
        d->stale = false;
    }
    b->stale = false;
    return WS_OK;
}

// Rebuild and upload descriptors, states and prefix tables from the domains
// (whose host copies are current: callers pull first).  The captured step
// stays valid unless the launch shapes changed.
static ws_status batch_upload(ws_batch *b) {
    if (batch_pull(b, b->last) != WS_OK) return WS_EHIP;
    std::vector<int> order;
    for (int sl = 0; sl < b->max; ++sl)
        if (b->slots[sl]) order.push_back(sl);
    const int n = (int)order.size();
    std::vector<BatchDesc> desc(n);
    b->h_state.assign(n, BatchState());
    std::vector<int> pre[5];
    for (int q = 0; q < 5; ++q) pre[q].assign(n + 1, 0);
    int maxK = 0, nred = 0;
    for (int k = 0; k < n; ++k) nred = std::max(nred, nred_of(b->slots[order[k]]));
    for (int k = 0; k < n; ++k) {
        ws_domain *d = b->slots[order[k]];
        if (d->solver != b->solver) {  // the batch's solve strategy (and layout) applies
            d->solver = b->solver;
            d->vdirty = true;
        }
        if (d->vdirty) {
            ws_status r = write_vtab(d);
            if (r != WS_OK) return r;
        }
        d->bidx = k;
        desc[k] = make_desc(d, b->sy);
        b->h_state[k].step = d->step;
        b->h_state[k].t = d->t;
        b->h_state[k].cur = d->cur;
        b->h_state[k].stop = d->stop;
        b->h_state[k].health = 0;
        const BatchDesc &D = desc[k];
        pre[0][k + 1] = pre[0][k] + D.sgx * D.sgy;
        pre[1][k + 1] = pre[1][k] + D.tgx * D.tgy;
        const dim3 sgc = strips_for(d, b->syc ? b->syc : b->sy, true);  // the corrector's one-wave grid
        pre[4][k + 1] = pre[4][k] + (int)(sgc.x * sgc.y);
        pre[2][k + 1] = pre[2][k] + (b->solver == WS_SOLVE_LU2                     ? solve2_waves(D.d.nx, D.d.ny)
                                     : b->solver == WS_SOLVE_LU && luw_waves(nred) ? luw_groups(D.d.nx, D.d.ny)
                                     : b->solver != WS_SOLVE_PCR && b->solver != WS_SOLVE_PCR_WAVE
                                         ? (D.d.ny + 63) / 64 + (D.d.nx + 63) / 64
                                         : D.nsys);
        pre[3][k + 1] = pre[3][k] + (D.makers ? (8 * D.d.gl * GHL + 255) / 256 : 0);
        maxK = D.K > maxK ? D.K : maxK;
    }
    if (n) {
        HIPCHK(hipMemcpy(b->d_desc, desc.data(), sizeof(BatchDesc) * n, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(b->d_state, b->h_state.data(), sizeof(BatchState) * n, hipMemcpyHostToDevice));
        for (int q = 0; q < 5; ++q)
            HIPCHK(hipMemcpy(b->d_pre[q], pre[q].data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice));
    }
    bool same = n == (int)b->order.size() && maxK == b->maxK && nred == b->nred;
    for (int q = 0; q < 5; ++q) same = same && pre[q][n] == b->total[q];
    if (!same) batch_drop_graph(b);
    b->order = order;
    b->maxK = maxK;
    b->nred = nred;
    for (int q = 0; q < 5; ++q) b->total[q] = pre[q][n];
    b->dirty = false;
    return WS_OK;
}

// The launches of one step for every domain of the batch.
static ws_status batch_step(ws_batch *b, hipStream_t st) {
    const int n = (int)b->order.size();
    if (b->total[3] > 0) {
        hipLaunchKernelGGL(kb_ghosts, dim3(b->total[3]), dim3(256), 0, st, b->d_desc, b->d_state, b->d_pre[3], n, 0);
        hipLaunchKernelGGL(kb_ghosts, dim3(b->total[3]), dim3(256), 0, st, b->d_desc, b->d_state, b->d_pre[3], n, 1);
    }
    for (int p = 0; p <= b->maxK; ++p) {
        // predictor pass: stencil_rows; corrector passes: their own height
        const int q = p > 0 ? 4 : 0, rows = p > 0 && b->syc ? b->syc : b->sy;
        const dim3 sg(b->total[q]), pg(b->total[2]);
#define L4(KERN) hipLaunchKernelGGL(KERN, sg, dim3(p > 0 ? 64 : 64 * SWG), 0, st, b->d_desc, b->d_state, b->d_pre[q], n, p)
        if (p > 0) SY_SWITCH(kb_stencil_c, rows, L4);
        else {
            SY_SWITCH(kb_stencil_e, rows, L4);
            SY_SWITCH(kb_stencil_p, rows, L4);
        }
#undef L4
        hipLaunchKernelGGL(kb_reduce, dim3(b->total[1]), dim3(NTB), 0, st, b->d_desc, b->d_state, b->d_pre[1], n, p);
        const size_t shm = sizeof(float4) * b->nred;
        if (b->solver == WS_SOLVE_LU2)
            hipLaunchKernelGGL(kb_lu2_solve, pg, dim3(64), 0, st, b->d_desc, b->d_state, b->d_pre[2], n, p);
        else if (b->solver == WS_SOLVE_LU)
            if (const int G = luw_waves(b->nred))
                hipLaunchKernelGGL(kb_luw_solve, pg, dim3(64 * G), 0, st, b->d_desc, b->d_state, b->d_pre[2], n, p);
            else
                hipLaunchKernelGGL(kb_lu_solve, pg, dim3(64), 0, st, b->d_desc, b->d_state, b->d_pre[2], n, p);
        else if (b->solver == WS_SOLVE_THOMAS)
            hipLaunchKernelGGL(kb_thomas, pg, dim3(64), 0, st, b->d_desc, b->d_state, b->d_pre[2], n, p);
        else if (b->solver == WS_SOLVE_PCR_WAVE && pcrw_fits(b->nred))  // (longer: the workgroup PCR, same bits)
            launch_pcrw_batch(b->nred, pg, st, b->d_desc, b->d_state, b->d_pre[2], n, p);
        else
            pcr_dispatch(b->pnt, pcr_epl(b->pnt, b->nred), [&](auto shape) {
                using S = decltype(shape);
                hipLaunchKernelGGL((kb_pcr<S::threads, S::epl>), pg, dim3(S::threads), shm, st, b->d_desc,
                                   b->d_state, b->d_pre[2], n, p);
            });
        hipLaunchKernelGGL(kb_expand, dim3(b->total[1]), dim3(NTB), 0, st, b->d_desc, b->d_state, b->d_pre[1], n, p);
    }
    hipLaunchKernelGGL(kb_finish, dim3((n + 255) / 256), dim3(256), 0, st, b->d_desc, b->d_state, n);
    HIPCHK(hipGetLastError());
    return WS_OK;
}

extern "C" size_t ws_batch_workspace_bytes(int32_t max_domains) {
    if (max_domains < 1) return 0;
    return batch_layout(max_domains, nullptr, nullptr);
}

extern "C" ws_status ws_batch_create(int32_t max_domains, void *workspace_dev, size_t bytes, ws_batch **out) {
    if (!out || max_domains < 1 || !workspace_dev) return fail(WS_EINVAL, "ws_batch_create: bad argument");
    if (((uintptr_t)workspace_dev & 255) != 0) return fail(WS_EINVAL, "ws_batch_create: workspace not 256-byte aligned");
    size_t o_state, o_pre;
    const size_t need = batch_layout(max_domains, &o_state, &o_pre);
    if (bytes < need) return fail(WS_ENOMEM, "ws_batch_create: workspace %zu < %zu bytes", bytes, need);
    ws_batch *b = new (std::nothrow) ws_batch();
    if (!b) return fail(WS_ENOMEM, "ws_batch_create: host allocation failed");
    char *base = (char *)workspace_dev;
    b->max = max_domains;
    b->d_desc = (BatchDesc *)base;
    b->d_state = (BatchState *)(base + o_state);
    const size_t c = align256(sizeof(int) * (size_t)(max_domains + 1));
    for (int q = 0; q < 5; ++q) b->d_pre[q] = (int *)(base + o_pre + q * c);
    b->slots.assign(max_domains, nullptr);
    *out = b;
    return WS_OK;
}

extern "C" ws_status ws_batch_destroy(ws_batch *b) {
    if (!b) return WS_OK;
    if (b->last) (void)hipStreamSynchronize(b->last);
    (void)batch_pull(b, b->last);
    for (ws_domain *d : b->slots)
        if (d) {
            d->batch = nullptr;
            d->stale = false;
        }
    batch_drop_graph(b);
    delete b;
    return WS_OK;
}

extern "C" ws_status ws_batch_attach(ws_batch *b, ws_domain *d, int32_t *slot) {
    if (!b || !d) return fail(WS_EINVAL, "ws_batch_attach: bad argument");
    if (d->batch) return fail(WS_EBUSY, "ws_batch_attach: domain already attached");
    if (d->tol_w > 0.0)
        return fail(WS_EINVAL, "ws_batch_attach: the corrector tolerance mode is single-domain only");
    // no sync: the tables are rebuilt (after a pull) by the next ws_batch_advance
    for (int sl = 0; sl < b->max; ++sl)
        if (!b->slots[sl]) {
            b->slots[sl] = d;
            d->batch = b;
            d->stale = false;
            d->stop = -1;
            b->dirty = true;
            if (slot) *slot = sl;
            return WS_OK;
        }
    return fail(WS_EBUSY, "ws_batch_attach: batch full (%d domains)", b->max);
}

extern "C" ws_status ws_batch_detach(ws_batch *b, int32_t slot) {
    if (!b || slot < 0 || slot >= b->max || !b->slots[slot]) return fail(WS_EINVAL, "ws_batch_detach: bad slot");
    if (batch_pull(b, b->last) != WS_OK) return WS_EHIP;
    ws_domain *d = b->slots[slot];
    d->batch = nullptr;
    d->stale = false;
    b->slots[slot] = nullptr;
    b->dirty = true;
    return WS_OK;
}

extern "C" ws_status ws_batch_set_stop(ws_batch *b, int32_t slot, int64_t stop_step) {
    if (!b || slot < 0 || slot >= b->max || !b->slots[slot]) return fail(WS_EINVAL, "ws_batch_set_stop: bad slot");
    ws_domain *d = b->slots[slot];
    d->stop = stop_step < 0 ? -1 : stop_step;  // uploaded (after a pull) by the next ws_batch_advance
    b->dirty = true;
    return WS_OK;
}

extern "C" ws_status ws_batch_status(ws_batch *b, int32_t slot, int64_t *step, double *t, int32_t *health) {
    if (!b || slot < 0 || slot >= b->max || !b->slots[slot]) return fail(WS_EINVAL, "ws_batch_status: bad slot");
    if (b->stale) return fail(WS_EBUSY, "ws_batch_status: call ws_batch_sync first");
    const ws_domain *d = b->slots[slot];
    if (step) *step = d->step;
    if (t) *t = d->t;
    if (health) *health = d->bhealth;
    return WS_OK;
}

extern "C" ws_status ws_batch_advance(ws_batch *b, int64_t nsteps, void *stream) {
    if (!b || nsteps < 0) return fail(WS_EINVAL, "ws_batch_advance: bad argument");
    hipStream_t st = (hipStream_t)stream;
    if (b->stale && b->last != st) {
        ws_status r = batch_pull(b, b->last);
        if (r != WS_OK) return r;
    }
    if (b->dirty) {
        if (b->last) HIPCHK(hipStreamSynchronize(b->last));
        ws_status r = batch_upload(b);
        if (r != WS_OK) return r;
    }
    if (b->order.empty() || nsteps == 0) return WS_OK;
    for (int sl : b->order) {
        ws_status r = ensure_factors(b->slots[sl], st);
        if (r != WS_OK) return r;
    }
    b->last = st;
    if (st != nullptr && (!b->exec || b->gstream != st)) {
        batch_drop_graph(b);
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
        ws_status r = batch_step(b, st);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(st, &g);
        if (r != WS_OK) {
            if (g) (void)hipGraphDestroy(g);
            return r;
        }
        if (e != hipSuccess) return fail(WS_EHIP, "ws_batch_advance: graph capture failed: %s", hipGetErrorString(e));
        b->graph = g;
        HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->gstream = st;
    }
    for (int64_t k = 0; k < nsteps; ++k) {
        if (b->exec) HIPCHK(hipGraphLaunch(b->exec, st));
        else {
            ws_status r = batch_step(b, st);
            if (r != WS_OK) return r;
        }
    }
    b->stale = true;
    for (int sl : b->order) b->slots[sl]->stale = true;
    return WS_OK;
}

extern "C" ws_status ws_batch_sync(ws_batch *b, void *stream) {
    if (!b) return fail(WS_EINVAL, "ws_batch_sync: NULL batch");
    return batch_pull(b, (hipStream_t)stream);
}

// ------------------------------------------------------------------ tuning
static bool tuning_ok(const ws_tuning *t) {
    return t && (t->stencil_rows == 8 || t->stencil_rows == 16 || t->stencil_rows == 24 ||
                 t->stencil_rows == 32 || t->stencil_rows == 48 || t->stencil_rows == 64) &&
           (t->pcr_threads == 64 || t->pcr_threads == 128 || t->pcr_threads == 256) &&
           (t->solver >= WS_SOLVE_PCR && t->solver <= WS_SOLVE_PCR_WAVE) &&
           (t->corrector_rows == 0 || t->corrector_rows == 8 || t->corrector_rows == 16 ||
            t->corrector_rows == 24 || t->corrector_rows == 32 || t->corrector_rows == 48 ||
            t->corrector_rows == 64);
}

extern "C" ws_status ws_get_tuning(const ws_domain *d, ws_tuning *out) {
    if (!d || !out) return fail(WS_EINVAL, "ws_get_tuning: bad argument");
    std::memset(out, 0, sizeof *out);
    out->stencil_rows = d->sy;
    out->pcr_threads = d->pnt;
    out->solver = d->solver;
    out->corrector_rows = d->syc;
    return WS_OK;
}

extern "C" ws_status ws_set_tuning(ws_domain *d, const ws_tuning *t) {
    if (!d || !tuning_ok(t)) return fail(WS_EINVAL, "ws_set_tuning: bad tuning");
    if (t->solver == WS_SOLVE_PCR_WAVE && !pcrw_fits(nred_of(d)))
        return fail(WS_EINVAL, "ws_set_tuning: reduced systems of %d unknowns are too long for the wave PCR (512)",
                    nred_of(d));
    d->sy = t->stencil_rows;
    d->syc = t->corrector_rows == t->stencil_rows ? 0 : t->corrector_rows;
    d->pnt = t->pcr_threads;
    if (d->solver != t->solver) batch_touch(d);  // argument blocks carry the solve layout
    d->solver = t->solver;
    return WS_OK;
}

extern "C" ws_status ws_batch_set_tuning(ws_batch *b, const ws_tuning *t) {
    if (!b || !tuning_ok(t)) return fail(WS_EINVAL, "ws_batch_set_tuning: bad tuning");
    const int syc = t->corrector_rows == t->stencil_rows ? 0 : t->corrector_rows;
    if (b->sy != t->stencil_rows || b->syc != syc || b->pnt != t->pcr_threads || b->solver != t->solver) {
        b->sy = t->stencil_rows;
        b->syc = syc;
        b->pnt = t->pcr_threads;
        b->solver = t->solver;
        b->dirty = true;
        b->total[0] = -1;  // launch shapes change: the captured step is rebuilt
    }
    return WS_OK;
}

static bool cache_lookup(const char *path, const ws_grid &g, ws_tuning *t) {
    if (!path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    int nx, ny, k, m, sy, pn, so, syc;
    bool hit = false;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        syc = 0;
        if (std::sscanf(line, "%d %d %d %d %d %d %d %d", &nx, &ny, &k, &m, &sy, &pn, &so, &syc) < 7) continue;
        if (nx == g.nx && ny == g.ny && k == g.n_corr && m == g.model) {
            t->stencil_rows = sy;
            t->pcr_threads = pn;
            t->solver = so;
            t->corrector_rows = syc;
            hit = tuning_ok(t);
        }
    }
    std::fclose(f);
    return hit;
}

extern "C" ws_status ws_tune(ws_domain *d, const char *cache_path, void *stream, ws_tuning *out) {
    if (!d || !out) return fail(WS_EINVAL, "ws_tune: bad argument");
    if (busy_check(d, "ws_tune") != WS_OK) return WS_EBUSY;
    ws_tuning best;
    std::memset(&best, 0, sizeof best);
    if (cache_lookup(cache_path, d->g, &best)) {
        ws_status r = ws_set_tuning(d, &best);
        if (r == WS_OK) *out = best;
        return r;
    }
    hipStream_t st = (hipStream_t)stream;
    // a corrector pass reads the current state and the corrector bases and
    // writes only the scratch estimate, the U*, V* increments and the solver
    // scratch: the state and history are untouched
    const Dom m = make_dom(d);
    StencilArgs sa;
    SolveArgs so;
    pass_args(d, m, false, d->cur, (int)((d->step + 1) % 3), d->g.n_corr > 0 ? 1 : 0, sa, so);
    sa.kind = 2;
    so.eta = d->st[(d->cur + 2) % 3][0];
    so.pout = d->st[(d->cur + 2) % 3][1];
    so.qout = d->st[(d->cur + 2) % 3][2];
    sa.eout = so.eta;
    so.sponge = 0;
    so.health = (int *)d->scal;  // keep the domain's health word out of the timing runs
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const int reps = 5;
    float best_p = 1e30f;
    best.stencil_rows = SY;
    best.pcr_threads = PCR_NT;
    best.solver = WS_SOLVE_PCR;
    // candidates are timed round-robin over three rounds and each keeps its
    // best round, so slow drift of the clock or of other load on the device
    // does not favour whichever candidate ran first
    // The next step's predictor pass (kind as that step takes it) rewrites
    // only what that step's own predictor rewrites before anything reads it:
    // the history level n, the corrector bases, the first estimate and the
    // increments; it reads the state and the older history levels only.
    StencilArgs sp;
    SolveArgs sop;
    pass_args(d, m, d->step + 1 <= 2, d->cur, (int)((d->step + 1) % 3), 0, sp, sop);
    const int rows[6] = {8, 16, 24, 32, 48, 64};
    float t_rows[2][6];
    for (int c = 0; c < 6; ++c) t_rows[0][c] = t_rows[1][c] = 1e30f;
    for (int c = 0; c < 6; ++c) {  // warm-up
        launch_stencil(d, rows[c], st, sp);
        launch_stencil(d, rows[c], st, sa);
    }
    for (int round = 0; round < 3; ++round)
        for (int kind = 0; kind < 2; ++kind)
            for (int c = 0; c < 6; ++c) {
                HIPCHK(hipEventRecord(e0, st));
                for (int k = 0; k < reps; ++k) launch_stencil(d, rows[c], st, kind ? sa : sp);
                HIPCHK(hipEventRecord(e1, st));
                HIPCHK(hipEventSynchronize(e1));
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                t_rows[kind][c] = ms < t_rows[kind][c] ? ms : t_rows[kind][c];
            }
    // one height for every pass unless separate heights save at least 2 % of
    // a step's stencil time (a single kernel instance keeps the per-kernel
    // accounting simple; smaller differences are within the timing noise)
    const int K = d->g.n_corr;
    int one = 0, cp = 0, cc = 0;
    for (int c = 1; c < 6; ++c) {
        if (t_rows[0][c] + K * t_rows[1][c] < t_rows[0][one] + K * t_rows[1][one]) one = c;
        if (t_rows[0][c] < t_rows[0][cp]) cp = c;
        if (t_rows[1][c] < t_rows[1][cc]) cc = c;
    }
    const float t_one = t_rows[0][one] + K * t_rows[1][one], t_two = t_rows[0][cp] + K * t_rows[1][cc];
    best.stencil_rows = rows[one];
    best.corrector_rows = 0;
    if (K > 0 && cp != cc && t_two < 0.98f * t_one) {
        best.stencil_rows = rows[cp];
        best.corrector_rows = rows[cc];
    }
    // Reduced-system strategies, each timed as the reduction (whose layout and
    // writes depend on the strategy: reduced equations, or right-hand sides
    // only for the factored solves) followed by the solve, `reps` times.
    const int nred = d->nu > d->nv ? d->nu : d->nv;
    const int threads[3] = {64, 128, 256};
    auto time_pairs = [&](const SolveArgs &sx, auto &&solve) -> float {
        hipLaunchKernelGGL(k_reduce, tiles(d), dim3(NT), 0, st, sx);  // warm-up
        solve();
        float total = 0.f;
        for (int k = 0; k < reps; ++k) {
            (void)hipEventRecord(e0, st);
            hipLaunchKernelGGL(k_reduce, tiles(d), dim3(NT), 0, st, sx);
            solve();
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            total += ms;
        }
        return total;
    };
    so.layout = 0;
    for (int c = 0; c < 3; ++c) {
        const float ms = time_pairs(so, [&] { launch_pcr(threads[c], nred, d->g.ny + d->g.nx, st, so); });
        if (ms < best_p) { best_p = ms; best.pcr_threads = threads[c]; best.solver = WS_SOLVE_PCR; }
    }
    if (pcrw_fits(nred)) {  // the wave form of PCR (same bits as the above)
        const float ms = time_pairs(so, [&] { launch_pcrw(nred, d->g.ny + d->g.nx, st, so); });
        if (ms < best_p) { best_p = ms; best.solver = WS_SOLVE_PCR_WAVE; }
    }
    {
        const int waves = (d->g.ny + 63) / 64 + (d->g.nx + 63) / 64;  // the sweep overwrites the equations
        const float ms = time_pairs(so, [&] { hipLaunchKernelGGL(k_thomas, dim3(waves), dim3(64), 0, st, so); });
        if (ms < best_p) { best_p = ms; best.solver = WS_SOLVE_THOMAS; }
    }
    {
        // factored solves: factors once (kept: they match the domain's current
        // bathymetry and boundaries), then only the right-hand-side sweeps
        const int keep = d->solver;
        SolveArgs s1 = so;
        s1.layout = 1;
        for (int sv : {WS_SOLVE_LU, WS_SOLVE_LU2}) {
            d->solver = sv;
            ws_status r = ensure_factors(d, st);
            if (r != WS_OK) {
                d->solver = keep;
                return r;
            }
            const float ms = time_pairs(s1, [&] { launch_reduced(d, st, s1); });
            if (ms < best_p) { best_p = ms; best.solver = sv; }
        }
        d->solver = keep;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(hipGetLastError());
    if (cache_path) {
        FILE *f = std::fopen(cache_path, "a");
        if (f) {
            std::fprintf(f, "%d %d %d %d %d %d %d %d\n", d->g.nx, d->g.ny, d->g.n_corr, d->g.model, best.stencil_rows,
                         best.pcr_threads, best.solver, best.corrector_rows);
            std::fclose(f);
        }
    }
    ws_status r = ws_set_tuning(d, &best);
    if (r == WS_OK) *out = best;
    return r;
}

// Batch autotuner: times the batched stencil of a corrector pass (pass 1:
// reads the states and corrector bases, writes only scratch) for every strip
// height, then the batched reduced solves for every thread count, and keeps
// the fastest.  Domains still in their start-up steps take no part.
extern "C" ws_status ws_batch_tune(ws_batch *b, void *stream, ws_tuning *out) {
    if (!b || !out) return fail(WS_EINVAL, "ws_batch_tune: bad argument");
    hipStream_t st = (hipStream_t)stream;
    ws_status r = batch_pull(b, b->last);
    if (r != WS_OK) return r;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    auto time_it = [&](auto &&launch) -> float {
        launch();
        (void)hipEventRecord(e0, st);
        for (int k = 0; k < 3; ++k) launch();
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        return ms;
    };
    const int rows[6] = {8, 16, 24, 32, 48, 64}, threads[3] = {64, 128, 256};
    int best_sy = b->sy, best_syc = b->syc, best_pnt = b->pnt, best_solver = WS_SOLVE_PCR;
    b->solver = WS_SOLVE_PCR;  // the PCR trials use the PCR prefix table
    float best = 1e30f, best_c = 1e30f, tp[6], tc[6];
    for (int c = 0; c < 6; ++c) tp[c] = tc[c] = 1e30f;
    b->syc = 0;
    for (int c = 0; c < 6; ++c) {
        b->sy = rows[c];
        b->dirty = true;
        if ((r = batch_upload(b)) != WS_OK) return r;
        const int n = (int)b->order.size();
        if (n == 0) break;
        // pass 0: each domain's next predictor (it rewrites only what that
        // step's predictor rewrites first); pass 1: a corrector (scratch only)
        float ms[2];
        for (int p = 0; p < 2; ++p)
            ms[p] = time_it([&] {
                const dim3 sg(b->total[p > 0 ? 4 : 0]);
#define L5(KERN) hipLaunchKernelGGL(KERN, sg, dim3(p > 0 ? 64 : 64 * SWG), 0, st, b->d_desc, b->d_state, b->d_pre[p > 0 ? 4 : 0], n, p)
                if (p > 0) SY_SWITCH(kb_stencil_c, b->sy, L5);
                else SY_SWITCH(kb_stencil_p, b->sy, L5);
#undef L5
            });
        tp[c] = ms[0];
        tc[c] = ms[1];
        if (ms[0] < best) { best = ms[0]; best_sy = rows[c]; }
        if (ms[1] < best_c) { best_c = ms[1]; best_syc = rows[c]; }
    }
    {
        // as in ws_tune: separate heights only when they save 2 % of a step's
        // stencil time (K = the batch's largest corrector count)
        int one = 0;
        for (int c = 1; c < 6; ++c)
            if (tp[c] + b->maxK * tc[c] < tp[one] + b->maxK * tc[one]) one = c;
        const bool two = b->maxK > 0 && best_sy != best_syc &&
                         best + b->maxK * best_c < 0.98f * (tp[one] + b->maxK * tc[one]);
        if (!two) best_sy = best_syc = rows[one];
    }
    b->sy = best_sy;
    b->syc = best_syc == best_sy ? 0 : best_syc;
    b->dirty = true;
    if ((r = batch_upload(b)) != WS_OK) return r;
    const int n = (int)b->order.size();
    best = 1e30f;
    if (n > 0) {
        // each strategy timed as the reduction (its layout depends on the
        // strategy) followed by the reduced solve
        auto reduce = [&] {
            hipLaunchKernelGGL(kb_reduce, dim3(b->total[1]), dim3(NTB), 0, st, b->d_desc, b->d_state, b->d_pre[1], n, 1);
        };
        for (int c = 0; c < 3; ++c) {
            const float ms = time_it([&] {
                reduce();
                const dim3 pg(b->total[2]);
                const size_t shm = sizeof(float4) * b->nred;
                pcr_dispatch(threads[c], pcr_epl(threads[c], b->nred), [&](auto shape) {
                    using S = decltype(shape);
                    hipLaunchKernelGGL((kb_pcr<S::threads, S::epl>), pg, dim3(S::threads), shm, st, b->d_desc,
                                       b->d_state, b->d_pre[2], n, 1);
                });
            });
            if (ms < best) { best = ms; best_pnt = threads[c]; }
        }
        if (pcrw_fits(b->nred)) {  // the wave form of PCR (the PCR prefix table)
            const float ms = time_it([&] {
                reduce();
                launch_pcrw_batch(b->nred, dim3(b->total[2]), st, b->d_desc, b->d_state, b->d_pre[2], n, 1);
            });
            if (ms < best) { best = ms; best_solver = WS_SOLVE_PCR_WAVE; }
        }
        // lane-per-system Thomas (its prefix table differs: rebuilt for the trial)
        b->solver = WS_SOLVE_THOMAS;  // trial
        b->dirty = true;
        if ((r = batch_upload(b)) != WS_OK) return r;
        float total = 0.f;
        for (int k = 0; k < 4; ++k) {
            (void)hipEventRecord(e0, st);
            reduce();
            hipLaunchKernelGGL(kb_thomas, dim3(b->total[2]), dim3(64), 0, st, b->d_desc, b->d_state, b->d_pre[2], n, 1);
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (k > 0) total += ms;
        }
        if (total < best) {
            best = total;
            best_solver = WS_SOLVE_THOMAS;
        }
        // factored solve: argument blocks with the interleaved layout, factors
        b->solver = WS_SOLVE_LU;  // trial
        b->dirty = true;
        if ((r = batch_upload(b)) != WS_OK) return r;
        for (int sl : b->order)
            if ((r = ensure_factors(b->slots[sl], st)) != WS_OK) return r;
        total = 0.f;
        for (int k = 0; k < 4; ++k) {
            (void)hipEventRecord(e0, st);
            reduce();
            if (const int G = luw_waves(b->nred))
                hipLaunchKernelGGL(kb_luw_solve, dim3(b->total[2]), dim3(64 * G), 0, st, b->d_desc, b->d_state,
                                   b->d_pre[2], n, 1);
            else
                hipLaunchKernelGGL(kb_lu_solve, dim3(b->total[2]), dim3(64), 0, st, b->d_desc, b->d_state,
                                   b->d_pre[2], n, 1);
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (k > 0) total += ms;
        }
        if (total < best) {
            best = total;
            best_solver = WS_SOLVE_LU;
        }
        b->solver = WS_SOLVE_LU2;  // trial
        b->dirty = true;
        if ((r = batch_upload(b)) != WS_OK) return r;
        for (int sl : b->order)
            if ((r = ensure_factors(b->slots[sl], st)) != WS_OK) return r;
        total = 0.f;
        for (int k = 0; k < 4; ++k) {
            (void)hipEventRecord(e0, st);
            reduce();
            hipLaunchKernelGGL(kb_lu2_solve, dim3(b->total[2]), dim3(64), 0, st, b->d_desc, b->d_state, b->d_pre[2], n, 1);
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (k > 0) total += ms;
        }
        if (total < best) best_solver = WS_SOLVE_LU2;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(hipGetLastError());
    b->pnt = best_pnt;
    b->solver = best_solver;
    b->total[0] = -1;  // the captured step is rebuilt with the chosen shapes
    b->dirty = true;
    std::memset(out, 0, sizeof *out);
    out->stencil_rows = b->sy;
    out->corrector_rows = b->syc;
    out->pcr_threads = b->pnt;
    out->solver = b->solver;
    return WS_OK;
}
