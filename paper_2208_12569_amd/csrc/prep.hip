// Field ingest and curl preparation.
//
// One streaming pass over the caller's Bx, By, Bz planes writes, per node, the
// record the tracer gathers: (Bx, By, Bz, Jx, Jy, Jz, 0, 0) in the compute type,
// J = curl B by second-order differences (central inside, the one-sided
// second-order formula on boundary nodes; the stencil of the paper's Eq. grad_B,
// Section 4; on a stretched axis the derivative of the quadratic through the same
// three nodes), or (Bx, By, Bz, 0) without the twist integrand. Interleaving the six
// values of a node in one aligned record lets one grid cell be fetched with 16
// vector loads from about 5 cache lines instead of 48 scalar gathers from six
// planes.
// The pass also reduces max |B|^2, the scale of the null-field test.
#include <float.h>

#include "fq_internal.h"

namespace fq {
namespace {

template <typename S>
__device__ __forceinline__ double ld(const S *p, int64_t i)
{
    return (double)p[i];
}

// d p / d axis at node (i,j,k) (stride = element distance along the axis).
template <typename S>
__device__ __forceinline__ double ddx(const S *p, int64_t q, int m, int n, int64_t stride,
                                      double inv_h)
{
    if (n < 3) return (ld(p, q - (int64_t)m * stride + stride) - ld(p, q - (int64_t)m * stride)) * inv_h;
    if (m == 0)
        return (-3.0 * ld(p, q) + 4.0 * ld(p, q + stride) - ld(p, q + 2 * stride)) * (0.5 * inv_h);
    if (m == n - 1)
        return (3.0 * ld(p, q) - 4.0 * ld(p, q - stride) + ld(p, q - 2 * stride)) * (0.5 * inv_h);
    return (ld(p, q + stride) - ld(p, q - stride)) * (0.5 * inv_h);
}

// The same on a stretched axis with node coordinates x: the derivative at node m of
// the quadratic through it and two other nodes (its neighbours inside, the next two
// inward on a boundary node), from the signed distances h1, h2 to them and the
// differences d1, d2 of p there: (d1 h2^2 - d2 h1^2) / (h1 h2 (h2 - h1)).
template <typename S>
__device__ __forceinline__ double ddx_s(const S *p, int64_t q, int m, int n, int64_t stride,
                                        const double *x)
{
    if (n < 3) return (ld(p, q - (int64_t)m * stride + stride) - ld(p, q - (int64_t)m * stride)) / (x[1] - x[0]);
    const int m1 = m == 0 ? 1 : (m == n - 1 ? n - 2 : m - 1);
    const int m2 = m == 0 ? 2 : (m == n - 1 ? n - 3 : m + 1);
    const double h1 = x[m1] - x[m], h2 = x[m2] - x[m];
    const double p0 = ld(p, q);
    const double d1 = ld(p, q + (int64_t)(m1 - m) * stride) - p0;
    const double d2 = ld(p, q + (int64_t)(m2 - m) * stride) - p0;
    return (d1 * h2 * h2 - d2 * h1 * h1) / (h1 * h2 * (h2 - h1));
}

template <typename S>
__device__ __forceinline__ double dax(const S *p, int64_t q, int m, int n, int64_t stride,
                                      double inv_h, const double *x)
{
    return x ? ddx_s(p, q, m, n, stride, x) : ddx(p, q, m, n, stride, inv_h);
}

template <typename T> struct V4;
template <> struct V4<float> { using t = float4; };
template <> struct V4<double> { using t = double4; };

template <typename S, typename T>
__global__ __launch_bounds__(256) void prep_kernel(const S *__restrict__ bx,
                                                   const S *__restrict__ by,
                                                   const S *__restrict__ bz, int nx, int ny,
                                                   int nz, double ihx, double ihy, double ihz,
                                                   const double *__restrict__ cx,
                                                   const double *__restrict__ cy,
                                                   const double *__restrict__ cz, int want_tw,
                                                   typename V4<T>::t *__restrict__ A,
                                                   float *__restrict__ bmax2)
{
    // a block takes a contiguous range of 256-node pieces of x rows (few blocks, so
    // the maximum of |B|^2 costs one atomic per block): the rows next to a row in y
    // are its own block's, and those next to it in z belong to blocks a fixed
    // distance away in the grid, which run at the same time on the same XCD, so the
    // neighbour reads of the curl differences mostly hit L2
    const int bxs = (nx + 255) / 256;
    const int64_t pieces = (int64_t)bxs * ny * nz;
    const int64_t nxy = (int64_t)nx * ny;
    const int64_t per = (pieces + gridDim.x - 1) / gridDim.x;
    const int64_t p_end = min(pieces, ((int64_t)blockIdx.x + 1) * per);
    float local = 0.0f;
    for (int64_t piece = (int64_t)blockIdx.x * per; piece < p_end; piece++) {
        const int64_t row = piece / bxs;
        const int i = (int)(piece - row * bxs) * 256 + (int)threadIdx.x;
        const int k = (int)(row / ny);
        const int j = (int)(row - (int64_t)k * ny);
        if (i >= nx) continue;
        const int64_t q = (int64_t)k * nxy + (int64_t)j * nx + i;
        const double Bx = ld(bx, q), By = ld(by, q), Bz = ld(bz, q);
        typename V4<T>::t a;
        a.x = (T)Bx;
        a.y = (T)By;
        a.z = (T)Bz;
        if (want_tw) {
            const double Jx = dax(bz, q, j, ny, nx, ihy, cy) - dax(by, q, k, nz, nxy, ihz, cz);
            const double Jy = dax(bx, q, k, nz, nxy, ihz, cz) - dax(bz, q, i, nx, 1, ihx, cx);
            const double Jz = dax(by, q, i, nx, 1, ihx, cx) - dax(bx, q, j, ny, nx, ihy, cy);
            a.w = (T)Jx;
            typename V4<T>::t c;
            c.x = (T)Jy;
            c.y = (T)Jz;
            c.z = (T)0;
            c.w = (T)0;
            A[2 * q] = a;
            A[2 * q + 1] = c;
        } else {
            a.w = (T)0;
            A[q] = a;
        }
        const float fb2 = (float)(Bx * Bx + By * By + Bz * Bz);
        if (fb2 > local) local = fb2;  // NaN compares false and is skipped
    }
    // block maximum, then one atomic per block (non-negative floats order like ints)
    for (int off = 32; off > 0; off >>= 1) {
        const float o = __shfl_xor(local, off);
        local = o > local ? o : local;
    }
    __shared__ float wmax[4];
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = local;
    __syncthreads();
    if (threadIdx.x == 0) {
        float m = 0.0f;
        for (int w = 0; w < (int)(blockDim.x + 63) / 64; w++) m = wmax[w] > m ? wmax[w] : m;
        if (m > 0.0f) {
            if (m > FLT_MAX) m = FLT_MAX;
            atomicMax((int *)bmax2, __float_as_int(m));
        }
    }
}

// Stretched grids: 1 / width of every cell of every axis (a uniform axis repeats
// 1 / spacing), the smallest width, and whether all widths are positive and finite
// and the stretched axes span the box given by origin and spacing. One block of 256.
__global__ __launch_bounds__(256) void geometry_kernel(GeoIn g, double *__restrict__ iw0,
                                                       double *__restrict__ iw1,
                                                       double *__restrict__ iw2, Geo *__restrict__ geo)
{
    double wmin = INFINITY;
    int bad = 0;
    for (int a = 0; a < 3; a++) {
        double *iw = a == 0 ? iw0 : (a == 1 ? iw1 : iw2);
        const double *x = g.coord[a];
        for (int c = (int)threadIdx.x; c < g.n[a] - 1; c += (int)blockDim.x) {
            const double w = x ? x[c + 1] - x[c] : g.spacing[a];
            const bool ok = w > 0.0 && w <= DBL_MAX;  // false for NaN
            iw[c] = ok ? 1.0 / w : NAN;
            if (ok) wmin = w < wmin ? w : wmin;
            bad |= !ok;
        }
    }
    // the first and last nodes of a stretched axis are the box's extent
    if (threadIdx.x == 0)
        for (int a = 0; a < 3; a++) {
            const double *x = g.coord[a];
            if (!x) continue;
            const double lo = g.origin[a], hi = g.origin[a] + (g.n[a] - 1) * g.spacing[a];
            const double tol = 1e-12 * (hi - lo);
            if (!(fabs(x[0] - lo) <= tol) || !(fabs(x[g.n[a] - 1] - hi) <= tol)) bad = 1;
        }
    __shared__ double smin[256];
    __shared__ int sbad[256];
    smin[threadIdx.x] = wmin;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            const double o = smin[threadIdx.x + h];
            smin[threadIdx.x] = o < smin[threadIdx.x] ? o : smin[threadIdx.x];
            sbad[threadIdx.x] |= sbad[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        geo->dref = smin[0];
        geo->bad = sbad[0];
        geo->pad = 0;
    }
}

__global__ void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename S, typename T>
hipError_t run_prep(const fq_field &f, int want_tw, void *A, float *bmax2, hipStream_t s)
{
    const int64_t pieces = ((f.n[0] + 255) / 256) * f.n[1] * f.n[2];
    const unsigned blocks = (unsigned)(pieces < 4096 ? pieces : 4096);
    hipLaunchKernelGGL((prep_kernel<S, T>), dim3(blocks), dim3(256), 0, s,
                       (const S *)f.b[0], (const S *)f.b[1], (const S *)f.b[2], (int)f.n[0],
                       (int)f.n[1], (int)f.n[2], 1.0 / f.spacing[0], 1.0 / f.spacing[1],
                       1.0 / f.spacing[2], f.coord[0], f.coord[1], f.coord[2], want_tw,
                       (typename V4<T>::t *)A, bmax2);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_geometry(const fq_field &f, double *const iw[3], Geo *geo, hipStream_t s)
{
    GeoIn g;
    for (int a = 0; a < 3; a++) {
        g.coord[a] = f.coord[a];
        g.n[a] = (int32_t)f.n[a];
        g.spacing[a] = f.spacing[a];
        g.origin[a] = f.origin[a];
    }
    hipLaunchKernelGGL(geometry_kernel, dim3(1), dim3(256), 0, s, g, iw[0], iw[1], iw[2], geo);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_prep(const fq_field &f, int prec, int want_tw, void *A, float *bmax2,
                       hipStream_t s)
{
    if (f.dtype == FQ_DT_F32) {
        return prec == FQ_PREC_F64 ? run_prep<float, double>(f, want_tw, A, bmax2, s)
                                   : run_prep<float, float>(f, want_tw, A, bmax2, s);
    }
    return prec == FQ_PREC_F64 ? run_prep<double, double>(f, want_tw, A, bmax2, s)
                               : run_prep<double, float>(f, want_tw, A, bmax2, s);
}

}  // namespace fq
