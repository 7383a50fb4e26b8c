// FP64 trilinear interpolation (Section 2.2, Eq. interp) straight from the caller's
// node planes, for the quantities kept in FP64: the normal fields entering Q and
// the field angles that send a line to the FP64 pass. Uniform and stretched
// rectilinear grids.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace fq {

struct Planes64 {
    const void *b[3];
    int32_t dtype;  // FQ_DT_F32 / FQ_DT_F64
    int32_t n[3];
    double origin[3], spacing[3];
    const double *coord[3];  // node coordinates of stretched axes (NULL = uniform axis)
};

// The cell of a stretched axis holding r: the last of the n nodes x at or below r,
// kept in [0, n-2] (bisection, Section 2.2). A point below the first node takes cell
// 0 and one at or above the last node cell n-2 (whose polynomial is then extended).
__host__ __device__ __forceinline__ int axis_cell(const double *x, int n, double r)
{
    int lo = 0, hi = n - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (x[mid] <= r) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Box extent and a typical cell width along axis a of a grid description (Planes64,
// MapJob: anything with n, origin, spacing and coord).
template <typename G>
__host__ __device__ __forceinline__ double axis_lo(const G &g, int a)
{
    return g.coord[a] ? g.coord[a][0] : g.origin[a];
}
template <typename G>
__host__ __device__ __forceinline__ double axis_hi(const G &g, int a)
{
    return g.coord[a] ? g.coord[a][g.n[a] - 1] : g.origin[a] + (g.n[a] - 1) * g.spacing[a];
}
template <typename G>
__host__ __device__ __forceinline__ double axis_width(const G &g, int a)
{
    return g.coord[a] ? (g.coord[a][g.n[a] - 1] - g.coord[a][0]) / (double)(g.n[a] - 1)
                      : g.spacing[a];
}

template <typename S>
__device__ __forceinline__ void interp64_t(const Planes64 &m, const double r[3], double B[3])
{
    const S *bx = (const S *)m.b[0], *by = (const S *)m.b[1], *bz = (const S *)m.b[2];
    int c[3];
    double t[3];
    for (int a = 0; a < 3; a++) {
        if (m.coord[a]) {
            const double *x = m.coord[a];
            const int ci = axis_cell(x, m.n[a], r[a]);
            c[a] = ci;
            t[a] = (r[a] - x[ci]) / (x[ci + 1] - x[ci]);
            continue;
        }
        const double g = (r[a] - m.origin[a]) / m.spacing[a];
        int ci = (int)floor(g);
        ci = ci < 0 ? 0 : (ci > m.n[a] - 2 ? m.n[a] - 2 : ci);
        c[a] = ci;
        t[a] = g - ci;
    }
    const int64_t sy = m.n[0], sz = (int64_t)m.n[0] * m.n[1];
    const int64_t base = c[2] * sz + c[1] * sy + c[0];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < 8; q++) {
        const int ix = q & 1, iy = (q >> 1) & 1, iz = (q >> 2) & 1;
        const double w = (ix ? t[0] : 1.0 - t[0]) * (iy ? t[1] : 1.0 - t[1]) *
                         (iz ? t[2] : 1.0 - t[2]);
        const int64_t o = base + ix + iy * sy + iz * sz;
        acc[0] += w * (double)bx[o];
        acc[1] += w * (double)by[o];
        acc[2] += w * (double)bz[o];
    }
    B[0] = acc[0];
    B[1] = acc[1];
    B[2] = acc[2];
}

__device__ __forceinline__ void interp64(const Planes64 &m, const double r[3], double B[3])
{
    if (m.dtype == 0) interp64_t<float>(m, r, B);
    else interp64_t<double>(m, r, B);
}

}  // namespace fq
