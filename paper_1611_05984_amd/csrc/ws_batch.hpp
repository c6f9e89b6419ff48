// ws_batch.hpp -- many independent domains advanced together.
//
// Every attached domain has a static descriptor (its grid, launch geometry
// and a table of the argument blocks of every pass variant) and a small
// device-side state (completed steps, time, current state buffer).  The pass
// bookkeeping that the single-domain path does on the host (Euler start-up,
// history slots, buffer rotation, ghost time level, sponge on the last pass)
// reduces to picking a table entry from that state on the device, so the
// launches of one step are identical from step to step and the step can be
// captured once in a hipGraph and replayed.  A workgroup copies its argument
// block from global memory before its first store (uniform addresses, so the
// copy is scalar loads into SGPRs, as for the single-domain kernels' own
// kernel-argument segment).  Each phase of a pass
// is one launch for all domains: workgroup b finds its domain by binary
// search in a prefix table of per-domain workgroup counts; domains still in
// their Euler start-up skip the corrector passes.  A last tiny kernel
// advances every domain's state.
#pragma once
#include "ws_kernels.hpp"

namespace ws {

struct BatchDesc {
    Dom d;                     // grid, depth, sides (wave-maker ghosts)
    const StencilArgs *sa;     // per-variant pass arguments (see variant())
    const SolveArgs *so;
    float *ghost[2];
    double dt;
    int K;                     // corrector passes of a full (AB3) step
    int sgx, sgy;              // stencil workgroup grid
    int tgx, tgy;              // solver tile grid
    int nsys;                  // reduced systems: ny + nx
    int makers;                // number of wave-maker sides
    int sgxc;                  // corrector stencil grid width (one-wave workgroups: the strip count)
    const int *health;         // the domain's health word
};

struct BatchState {
    long long step;            // completed steps since (re)start
    long long stop;            // pause once step reaches it (-1: no limit)
    double t;
    int cur;                   // state buffer of the current state
    int health;                // copy of the domain's health word after the step
};

__device__ __forceinline__ bool paused(const BatchState &S) { return S.stop >= 0 && S.step >= S.stop; }

// Argument-table entry of pass p of the step a domain takes next, or -1 when
// the domain has no such pass (correctors of the Euler start-up steps) or is
// paused at its step limit.
// Entries 0..8: Euler steps by (state buffer, step mod 3); then full steps by
// (state buffer, step mod 3, pass).
__device__ __forceinline__ int variant(const BatchDesc &D, const BatchState &S, int p) {
    if (paused(S)) return -1;
    const long long s = S.step + 1;
    const int sm = (int)(s % 3), key = S.cur * 3 + sm;
    if (s <= 2) return p == 0 ? key : -1;
    return p <= D.K ? 9 + key * (D.K + 1) + p : -1;
}

// Copy of a block of kernel parameters held in global memory, read through the
// constant address space: workgroup-uniform scalar loads into SGPRs (valid
// only for memory no kernel of the launch writes).
template <class T> __device__ __forceinline__ T load_params(const T *p) {
    static_assert(sizeof(T) % 4 == 0, "parameter blocks are whole dwords");
    T r;
    const __attribute__((address_space(4))) unsigned *src = (const __attribute__((address_space(4))) unsigned *)p;
    unsigned *dst = reinterpret_cast<unsigned *>(&r);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = src[i];
    return r;
}

__device__ __forceinline__ int find_dom(const int *prefix, int ndom, int b) {
    int lo = 0, hi = ndom;  // prefix[lo] <= b < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

// KIND: 0 for the predictor pass of domains in their Euler start-up, 1 for
// that of domains taking full steps (each domain's predictor runs in exactly
// one of the two launches), 2 for the corrector passes.  The bodies are the
// single-domain kernels' own, so both give the same bits.
template <int SYT, int KIND>
__device__ __forceinline__ void kb_stencil_body(const BatchDesc *__restrict__ descs, const BatchState *__restrict__ states,
                                                const int *__restrict__ prefix, int ndom, int p) {
    // XCD-aware order over all strips of all domains (as in k_stencil_*)
    const int b = xcd_order(blockIdx.x, gridDim.x), dm = find_dom(prefix, ndom, b);
    const BatchDesc &D = descs[dm];
    const BatchState &S = states[dm];
    if (KIND < 2 && (S.step + 1 <= 2) != (KIND == 0)) return;  // the other predictor launch's domain
    const int v = variant(D, S, p);
    if (v < 0) return;
    const int local = b - prefix[dm];
    const StencilArgs A = load_params(D.sa + v);
    if constexpr (KIND == 2)  // one-wave workgroups, as the single-domain corrector
        stencil_body<SYT, 2, true>(A, local % D.sgxc, local / D.sgxc);
    else
        stencil_body<SYT, KIND>(A, local % D.sgx, local / D.sgx);
}
template <int SYT>
__global__ __launch_bounds__(64 * SWG) __attribute__((amdgpu_waves_per_eu(4))) void kb_stencil_e(const BatchDesc *__restrict__ descs,
                                                         const BatchState *__restrict__ states,
                                                         const int *__restrict__ prefix, int ndom, int p) {
    kb_stencil_body<SYT, 0>(descs, states, prefix, ndom, p);
}
template <int SYT>
__global__ __launch_bounds__(64 * SWG) __attribute__((amdgpu_waves_per_eu(4))) void kb_stencil_p(const BatchDesc *__restrict__ descs,
                                                         const BatchState *__restrict__ states,
                                                         const int *__restrict__ prefix, int ndom, int p) {
    kb_stencil_body<SYT, 1>(descs, states, prefix, ndom, p);
}
template <int SYT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void kb_stencil_c(const BatchDesc *__restrict__ descs,
                                                         const BatchState *__restrict__ states,
                                                         const int *__restrict__ prefix, int ndom, int p) {
    kb_stencil_body<SYT, 2>(descs, states, prefix, ndom, p);
}

// The batch's tile kernels run two-wave workgroups (NTB threads): over many
// small domains that is 2.6 % faster than the single-domain kernels' four
// waves, which are 9 % faster on one large domain.  The same arithmetic per
// cell either way.
__global__ __launch_bounds__(NTB) void kb_reduce(const BatchDesc *__restrict__ descs,
                                                const BatchState *__restrict__ states,
                                                const int *__restrict__ prefix, int ndom, int p) {
    __shared__ SolveTile s;
    const int b = blockIdx.x, dm = find_dom(prefix, ndom, b);
    const BatchDesc &D = descs[dm];
    const int v = variant(D, states[dm], p);
    if (v < 0) return;
    const int local = b - prefix[dm];
    const SolveArgs A = load_params(D.so + v);
    reduce_body<NTB>(A, s, local % D.tgx, local / D.tgx);
}

template <int PNT, int EPL>
__global__ __launch_bounds__(PNT) void kb_pcr(const BatchDesc *__restrict__ descs,
                                                 const BatchState *__restrict__ states,
                                                 const int *__restrict__ prefix, int ndom, int p) {
    extern __shared__ float4 buf[];
    const int b = blockIdx.x, dm = find_dom(prefix, ndom, b);
    const BatchDesc &D = descs[dm];
    const int v = variant(D, states[dm], p);
    if (v < 0) return;
    const SolveArgs *g = D.so + v;  // only the fields the solve needs
    const int sys = b - prefix[dm], ny = load_params(&g->d.ny);
    if (sys < ny) {
        const int N = load_params(&g->d.nu);
        pcr_solve<PNT, EPL>(N, load_params(&g->redx) + (size_t)sys * N, load_params(&g->solx) + (size_t)sys * N, buf);
    } else {
        const int N = load_params(&g->d.nv);
        pcr_solve<PNT, EPL>(N, load_params(&g->redy) + (size_t)(sys - ny) * N, load_params(&g->soly) + (size_t)(sys - ny) * N,
                  buf);
    }
}

// The wave form of PCR over a batch: one wave per system, as k_pcrw; EPL is
// the batch's largest (at most 8: systems of up to 512 unknowns).
template <int EPL>
__global__ __launch_bounds__(64) void kb_pcrw(const BatchDesc *__restrict__ descs,
                                              const BatchState *__restrict__ states,
                                              const int *__restrict__ prefix, int ndom, int p) {
    const int b = blockIdx.x, dm = find_dom(prefix, ndom, b);
    const BatchDesc &D = descs[dm];
    const int v = variant(D, states[dm], p);
    if (v < 0) return;
    const SolveArgs *g = D.so + v;
    const int sys = b - prefix[dm], ny = load_params(&g->d.ny);
    if (sys < ny) {
        const int N = load_params(&g->d.nu);
        pcrw_solve<EPL>(N, load_params(&g->redx) + (size_t)sys * N, load_params(&g->solx) + (size_t)sys * N);
    } else {
        const int N = load_params(&g->d.nv);
        pcrw_solve<EPL>(N, load_params(&g->redy) + (size_t)(sys - ny) * N, load_params(&g->soly) + (size_t)(sys - ny) * N);
    }
}

__global__ __launch_bounds__(NTB) void kb_expand(const BatchDesc *__restrict__ descs,
                                                const BatchState *__restrict__ states,
                                                const int *__restrict__ prefix, int ndom, int p) {
    __shared__ SolveTile s;
    const int b = blockIdx.x, dm = find_dom(prefix, ndom, b);
    const BatchDesc &D = descs[dm];
    const int v = variant(D, states[dm], p);
    if (v < 0) return;
    const int local = b - prefix[dm];
    const SolveArgs A = load_params(D.so + v);
    expand_body<NTB>(A, s, local % D.tgx, local / D.tgx);
}

// Reduced systems by lane-per-system Thomas: workgroup (one wave) b - prefix
// of a domain takes row systems first, then column systems.
__global__ __launch_bounds__(64) void kb_thomas(const BatchDesc *__restrict__ descs,
                                                const BatchState *__restrict__ states,
                                                const int *__restrict__ prefix, int ndom, int p) {
    const int b = blockIdx.x, dm = find_dom(prefix, ndom, b);
    const BatchDesc &D = descs[dm];
    const int v = variant(D, states[dm], p);
    if (v < 0) return;
    const SolveArgs *g = D.so + v;
    const int wave = b - prefix[dm], lane = threadIdx.x;
    const int ny = load_params(&g->d.ny), nx = load_params(&g->d.nx), xw = (ny + 63) / 64;
    if (wave < xw) {
        const int sys = wave * 64 + lane, N = load_params(&g->d.nu);
        if (sys < ny) thomas_lane(N, load_params(&g->redx) + (size_t)sys * N, load_params(&g->solx) + (size_t)sys * N);
    } else {
        const int sys = (wave - xw) * 64 + lane, N = load_params(&g->d.nv);
        if (sys < nx) thomas_lane(N, load_params(&g->redy) + (size_t)sys * N, load_params(&g->soly) + (size_t)sys * N);
    }
}

// Factored reduced solves (layout 1): one wave per 64 systems of a domain.
__global__ __launch_bounds__(64) void kb_lu_solve(const BatchDesc *__restrict__ descs,
                                                  const BatchState *__restrict__ states,
                                                  const int *__restrict__ prefix, int ndom, int p) {
    const int b = blockIdx.x, dm = find_dom(prefix, ndom, b);
    const BatchDesc &D = descs[dm];
    const int v = variant(D, states[dm], p);
    if (v < 0) return;
    const SolveArgs A = load_params(D.so + v);
    lu_solve_body(A, b - prefix[dm], threadIdx.x);
}

// One-ended factored solves, workgroup form (see luw_solve_body); every
// workgroup of a paused domain leaves at once, before any barrier.
__global__ __launch_bounds__(64 * LUW_MAX) void kb_luw_solve(const BatchDesc *__restrict__ descs,
                                                             const BatchState *__restrict__ states,
                                                             const int *__restrict__ prefix, int ndom, int p) {
    __shared__ float slot[64];
    const int b = blockIdx.x, dm = find_dom(prefix, ndom, b);
    const BatchDesc &D = descs[dm];
    const int v = variant(D, states[dm], p);
    if (v < 0) return;
    const SolveArgs A = load_params(D.so + v);
    luw_solve_body(A, b - prefix[dm], slot);
}

// Two-ended factored solves: lane pairs per system (see lu2_solve_body).
__global__ __launch_bounds__(64) void kb_lu2_solve(const BatchDesc *__restrict__ descs,
                                                   const BatchState *__restrict__ states,
                                                   const int *__restrict__ prefix, int ndom, int p) {
    const int b = blockIdx.x, dm = find_dom(prefix, ndom, b);
    const BatchDesc &D = descs[dm];
    const int v = variant(D, states[dm], p);
    if (v < 0) return;
    const SolveArgs A = load_params(D.so + v);
    lu2_solve_body(A, b - prefix[dm], threadIdx.x);
}

// Wave-maker ghosts of t^n (which = 0) and t^{n+1} (which = 1); 256 threads
// per block, 8 gl GHL threads per domain with wave makers.
__global__ void kb_ghosts(const BatchDesc *descs, const BatchState *states, const int *prefix, int ndom,
                          int which) {
    const int b = blockIdx.x, dm = find_dom(prefix, ndom, b);
    const BatchDesc &D = descs[dm];
    if (!D.makers || paused(states[dm])) return;
    const int k = (b - prefix[dm]) * blockDim.x + threadIdx.x;
    if (k >= 8 * D.d.gl * GHL) return;  // whole lane groups (8 gl GHL is a multiple of GHL)
    const double t = states[dm].t + (which ? D.dt : 0.0);
    ghosts_body(D.d, D.ghost[which], t, k);
}

// Completes the step of every domain: buffer of the final estimate, step, time.
__global__ void kb_finish(const BatchDesc *descs, BatchState *states, int ndom) {
    const int dm = blockIdx.x * blockDim.x + threadIdx.x;
    if (dm >= ndom) return;
    BatchState S = states[dm];
    S.health = *descs[dm].health;
    if (paused(S)) {
        states[dm] = S;
        return;
    }
    const long long s = S.step + 1;
    const int K = s <= 2 ? 0 : descs[dm].K;
    const int b = (S.cur + 1) % 3, c = (S.cur + 2) % 3;
    S.cur = K == 0 ? b : ((K & 1) ? c : b);
    S.step = s;
    S.t = S.t + descs[dm].dt;
    states[dm] = S;
}

}  // namespace ws
