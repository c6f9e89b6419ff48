// ws_probe.hip -- HBM streaming ceilings for the measurement of the time step
// (libwsprobe.so; only the benchmark loads it).  Each kernel streams NR input
// fields and NW output fields of `rows` rows of `pitch` floats (structure of
// arrays, one field stride apart), with the access shape of the solver's
// stencils: one wave64 owns a 64-column strip, each lane loads and stores one
// dword per field per row, and the wave walks `wrows` consecutive rows.  A
// plain 16-byte-per-lane copy gives the runtime-independent copy ceiling
// (and, under the profiler, the scale of the HBM byte counters).
#include <hip/hip_runtime.h>

#include <cstddef>

namespace {

template <int NR, int NW>
__global__ __launch_bounds__(64) void k_stream(const float *__restrict__ in, float *__restrict__ out,
                                               size_t fstride, int pitch, int rows, int wrows) {
    const int strips = pitch / 64;
    const int s = blockIdx.x % strips, rb = blockIdx.x / strips;
    const int col = s * 64 + (int)threadIdx.x;
    const int r0 = rb * wrows, r1 = min(rows, r0 + wrows);
    for (int r = r0; r < r1; ++r) {
        const size_t o = (size_t)r * pitch + col;
        float v[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) v[k] = __builtin_nontemporal_load(in + k * fstride + o);
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < NR; ++k) acc += v[k];
#pragma unroll
        for (int k = 0; k < NW; ++k) out[k * fstride + o] = acc + (float)k;
    }
}

// The predictor's fields with its history levels, bases and increments
// packed per cell: reads 4 scalar fields, one 3-float and one 2-float level
// (n-1), one 3-float level (n-2); writes one 3-float and one 2-float level
// (n), 3-float bases, the surface and a 2-float increment pair.  PACKC: the
// corrector's: 4 scalar fields and 3-float bases read, the surface and the
// increment pair written.
struct f3 { float x, y, z; };
template <bool PRED>
__global__ __launch_bounds__(64) void k_stream_packed(const float *__restrict__ in, float *__restrict__ out,
                                                      size_t fstride, int pitch, int rows, int wrows) {
    const int strips = pitch / 64;
    const int s = blockIdx.x % strips, rb = blockIdx.x / strips;
    const int col = s * 64 + (int)threadIdx.x;
    const int r0 = rb * wrows, r1 = min(rows, r0 + wrows);
    const float *sc = in;                                             // 4 scalar fields
    const f3 *l1a = reinterpret_cast<const f3 *>(in + 4 * fstride);   // 3 floats a cell
    const float2 *l1b = reinterpret_cast<const float2 *>(in + 7 * fstride);
    const f3 *l2a = reinterpret_cast<const f3 *>(in + 9 * fstride);
    f3 *o0a = reinterpret_cast<f3 *>(out);
    float2 *o0b = reinterpret_cast<float2 *>(out + 3 * fstride);
    f3 *oS = reinterpret_cast<f3 *>(out + 5 * fstride);
    float *oe = out + 8 * fstride;
    float2 *ouv = reinterpret_cast<float2 *>(out + 9 * fstride);
    for (int r = r0; r < r1; ++r) {
        const size_t o = (size_t)r * pitch + col;
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < 4; ++k) acc += __builtin_nontemporal_load(sc + k * fstride + o);
        if (PRED) {
            const f3 a = l1a[o], c = l2a[o];
            const float2 b = l1b[o];
            acc += a.x + a.y + a.z + b.x + b.y + c.x + c.y + c.z;
            o0a[o] = f3{acc, acc + 1.f, acc + 2.f};
            o0b[o] = make_float2(acc + 3.f, acc + 4.f);
        } else {
            const f3 a = l1a[o];
            acc += a.x + a.y + a.z;
        }
        if (PRED) oS[o] = f3{acc + 5.f, acc + 6.f, acc + 7.f};
        oe[o] = acc + 8.f;
        ouv[o] = make_float2(acc + 9.f, acc + 10.f);
    }
}

__global__ __launch_bounds__(256) void k_copy4(const float4 *__restrict__ in, float4 *__restrict__ out, size_t n4) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x)
        out[i] = in[i];
}

}  // namespace

// kind 0: copy with 16-byte lanes of one field (in -> out, rows * pitch floats);
// kind 1: 7 fields read, 3 written (the corrector stencil's compulsory fields);
// kind 2: 12 fields read, 11 written (the predictor stencil's);
// kind 3: the predictor's 23 words in 12 packed streams; kind 4: the
// corrector's 10 words in 5 streams (both need room for 12 fields in `in` and
// 11 in `out`).  Otherwise `in` must hold NR fields and `out` NW fields of
// fstride = rows * pitch
// floats each; pitch a multiple of 64.  Launches `reps` times on `stream`
// and returns the mean milliseconds per launch in *ms (HIP events).
// Returns 0, or -1 for a bad argument, -2 for a HIP error.
extern "C" int wsp_stream(int kind, const float *in, float *out, int pitch, int rows, int wrows, int reps,
                          void *stream, float *ms) {
    if (!in || !out || !ms || pitch <= 0 || pitch % 64 || rows <= 0 || wrows <= 0 || reps <= 0 || kind < 0 ||
        kind > 4)
        return -1;
    hipStream_t st = (hipStream_t)stream;
    const size_t fstride = (size_t)rows * pitch;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -2;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return -2; }
    const unsigned blocks = (unsigned)((pitch / 64) * ((rows + wrows - 1) / wrows));
    auto launch = [&]() {
        if (kind == 0) {
            const size_t n4 = fstride / 4;
            hipLaunchKernelGGL(k_copy4, dim3(4096), dim3(256), 0, st, (const float4 *)in, (float4 *)out, n4);
        } else if (kind == 1) {
            hipLaunchKernelGGL((k_stream<7, 3>), dim3(blocks), dim3(64), 0, st, in, out, fstride, pitch, rows, wrows);
        } else if (kind == 2) {
            hipLaunchKernelGGL((k_stream<12, 11>), dim3(blocks), dim3(64), 0, st, in, out, fstride, pitch, rows, wrows);
        } else if (kind == 3) {
            hipLaunchKernelGGL((k_stream_packed<true>), dim3(blocks), dim3(64), 0, st, in, out, fstride, pitch, rows,
                               wrows);
        } else {
            hipLaunchKernelGGL((k_stream_packed<false>), dim3(blocks), dim3(64), 0, st, in, out, fstride, pitch, rows,
                               wrows);
        }
    };
    launch();  // warm-up
    int rc = 0;
    if (hipEventRecord(e0, st) != hipSuccess) rc = -2;
    for (int k = 0; k < reps && rc == 0; ++k) launch();
    if (rc == 0 && hipEventRecord(e1, st) != hipSuccess) rc = -2;
    if (rc == 0 && hipEventSynchronize(e1) != hipSuccess) rc = -2;
    if (rc == 0 && hipGetLastError() != hipSuccess) rc = -2;
    float t = 0.f;
    if (rc == 0 && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = -2;
    *ms = t / reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}
