// Gather microbenchmark: the tracer's cell fetches without its arithmetic.
//
// Every lane walks from cell to neighbouring cell through a node-record array laid
// out as the tracer's (8 FP32 values per node: B and curl B), fetching the 8 corner
// records of each cell with the same 16 vector loads. The next cell depends on the
// values just loaded (one fetch in flight per lane, as in the tracer, where the next
// cell follows from the field), and the walks look like field lines: a persistent
// direction biased upwards, the lanes of a wave starting on neighbouring cells of the
// bottom face. Two kinds of walk: incoherent (each lane draws its own moves, from a
// 2 x 2 patch of start cells) and coherent (the 64 lanes of a wave start on an 8 x 8
// patch and take the same moves, as neighbouring field lines do before they part).
// The rate of fetches x 192 useful bytes (24 values of B and curl B at 8 corners) is
// the gather roofline the tracer is measured against. A second kernel measures the FP32 FMA
// rate, the arithmetic ceiling of the same lanes.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint32_t mix(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

__global__ __launch_bounds__(256) void gather_walk_kernel(const float4 *__restrict__ rec, int nx,
                                                          int ny, int nz, int steps, uint32_t seed,
                                                          int coherent, float *__restrict__ sink)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int64_t wave = g >> 6;
    // a wave starts on a 2 x 2 (incoherent) or 8 x 8 (coherent) patch of bottom cells;
    // patches tile the bottom face
    const int side = coherent ? 8 : 2;
    const int px = (nx - 1) / side, py = (ny - 1) / side;
    const int64_t patch = (wave * 7919) % ((int64_t)px * py);
    int cx = (int)(patch % px) * side + (coherent ? (lane & 7) : (lane & 1));
    int cy = (int)(patch / px) * side + (coherent ? (lane >> 3) : ((lane >> 1) & 1));
    int cz = 0;
    uint32_t r = mix((uint32_t)(coherent ? wave : g) ^ seed);
    // persistent direction: weights for x, y and an upward-biased z (in 1/256)
    int wx = (int)(r & 127), wy = (int)((r >> 7) & 127), wz = 64 + (int)((r >> 14) & 127);
    int sxn = (r >> 21) & 1 ? 1 : -1, syn = (r >> 22) & 1 ? 1 : -1, szn = 1;
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    float acc = 0.0f;
    for (int s = 0; s < steps; s++) {
        const int64_t base = (int64_t)cz * sz + (int64_t)cy * sy + cx;
        float v = 0.0f;
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const int64_t o = base + ((q & 1) ? 1 : 0) + ((q & 2) ? sy : 0) + ((q & 4) ? sz : 0);
            const float4 a = rec[2 * o];
            const float4 c = rec[2 * o + 1];
            v += a.x + a.y + a.z + a.w + c.x + c.y;
        }
        acc += v;
        // next cell: an axis drawn with the lane's weights, perturbed by the data (the
        // first lane's, in a coherent walk)
        r = mix(r ^ __float_as_uint(coherent ? __shfl(v, 0) : v));
        const int pick = (int)(r % (uint32_t)(wx + wy + wz));
        if (pick < wx) {
            cx += sxn;
            if (cx < 0 || cx > nx - 2) { sxn = -sxn; cx += 2 * sxn; }
        } else if (pick < wx + wy) {
            cy += syn;
            if (cy < 0 || cy > ny - 2) { syn = -syn; cy += 2 * syn; }
        } else {
            cz += szn;
            if (cz < 0 || cz > nz - 2) { szn = -szn; cz += 2 * szn; }
        }
        cx = cx < 0 ? 0 : (cx > nx - 2 ? nx - 2 : cx);
        cy = cy < 0 ? 0 : (cy > ny - 2 ? ny - 2 : cy);
        cz = cz < 0 ? 0 : (cz > nz - 2 ? nz - 2 : cz);
    }
    sink[g] = acc;
}

// FP32 FMA rate: each lane runs `iters` iterations of 8 independent FMA chains, enough
// independent work to cover the FMA latency; the sum is stored so that the chains
// stay. Built like the library (packed FP32 instructions off): one FMA per lane per
// instruction.
__global__ __launch_bounds__(256) void fma_kernel(int iters, float a, float b, float *__restrict__ sink)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float x[8];
#pragma unroll
    for (int q = 0; q < 8; q++) x[q] = (float)threadIdx.x * 1e-3f + (float)q;
#pragma unroll 4
    for (int i = 0; i < iters; i++) {
#pragma unroll
        for (int q = 0; q < 8; q++) x[q] = fmaf(x[q], a, b);
    }
    float acc = 0.0f;
#pragma unroll
    for (int q = 0; q < 8; q++) acc += x[q];
    sink[g] = acc;
}

}  // namespace

extern "C" {

// records: nx*ny*nz nodes x 8 floats (device); lanes = blocks * 256; steps per lane;
// coherent: nonzero for the coherent walk. Asynchronous on `stream`; returns a
// hipError_t code.
int fqgb_walk(const void *records, int nx, int ny, int nz, int steps, int blocks, uint32_t seed,
              int coherent, float *sink, void *stream)
{
    if (!records || !sink || nx < 17 || ny < 17 || nz < 3 || steps < 1 || blocks < 1) return 1;
    hipLaunchKernelGGL(gather_walk_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       (const float4 *)records, nx, ny, nz, steps, seed, coherent, sink);
    return (int)hipGetLastError();
}

// FMA chains: lanes = blocks * 256, each `iters` x 8 FMAs (16 flops per iteration);
// sink: blocks * 256 floats (device). Asynchronous on `stream`; returns a hipError_t
// code.
int fqgb_fma(int iters, int blocks, float *sink, void *stream)
{
    if (!sink || iters < 1 || blocks < 1) return 1;
    hipLaunchKernelGGL(fma_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, iters,
                       0.999999f, 1e-7f, sink);
    return (int)hipGetLastError();
}

}  // extern "C"
