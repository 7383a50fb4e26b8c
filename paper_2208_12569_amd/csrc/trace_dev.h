// Device helpers shared by the tracer and its adjoint: node-record fetch, job-table
// decoding and seed positions.
#pragma once

#include "fq_internal.h"
#include "trace_core.h"

namespace fq {
namespace dev {

template <typename T> struct V4;
template <> struct V4<float> { using t = float4; };
template <> struct V4<double> { using t = double4; };

// Pointers read from the job table are generic; marking them as global memory
// (address space 1) makes the compiler emit global instead of flat loads/stores.
#if defined(__HIP_DEVICE_COMPILE__)
#define FQ_GLOBAL __attribute__((address_space(1)))
#else
#define FQ_GLOBAL
#endif
template <typename P> __device__ __forceinline__ FQ_GLOBAL P *gptr(P *p)
{
    return (FQ_GLOBAL P *)p;
}
template <typename P> __device__ __forceinline__ const FQ_GLOBAL P *gptr(const P *p)
{
    return (const FQ_GLOBAL P *)p;
}

// Fetch one cell: 8 corner records of type S, turned into monomial coefficients of
// type T. WIDE records hold 8 values (Bx, By, Bz, Jx | Jy, Jz, 0, 0): both halves of a
// corner come from one 32-byte (FP32) record, so a cell touches about 5 cache lines;
// narrow records are (Bx, By, Bz, 0). TW: build the curl coefficients too.
template <typename T, typename S, bool TW, bool WIDE = TW>
__device__ __forceinline__ void load_cell(const void *nodes, int nx, int ny, int cx, int cy,
                                          int cz, T cb[3][8], T cj[3][8])
{
    const FQ_GLOBAL typename V4<S>::t *A = gptr((const typename V4<S>::t *)nodes);
    const int64_t sx = 1, sy = nx, sz = (int64_t)nx * ny;
    const int64_t base = (int64_t)cz * sz + (int64_t)cy * sy + cx;
    T f[6][8];
#pragma unroll
    for (int q = 0; q < 8; q++) {
        const int64_t o = base + ((q & 1) ? sx : 0) + ((q & 2) ? sy : 0) + ((q & 4) ? sz : 0);
        const typename V4<S>::t a = A[WIDE ? 2 * o : o];
        f[0][q] = (T)a.x;
        f[1][q] = (T)a.y;
        f[2][q] = (T)a.z;
        f[3][q] = (T)a.w;
        if (TW) {
            const typename V4<S>::t c = A[2 * o + 1];
            f[4][q] = (T)c.x;
            f[5][q] = (T)c.y;
        }
    }
#pragma unroll
    for (int m = 0; m < 3; m++) coeffs<T>(f[m], cb[m]);
    if (TW) {
#pragma unroll
        for (int m = 0; m < 3; m++) coeffs<T>(f[3 + m], cj[m]);
    }
}

__device__ __forceinline__ unsigned long long shfl_u64(unsigned long long v, int src)
{
    unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
    lo = __shfl(lo, src);
    hi = __shfl(hi, src);
    return ((unsigned long long)hi << 32) | lo;
}

// Lines of a job that exist now (a rotated-S0 job is sized on the device).
__device__ __forceinline__ int64_t live_lines(const TraceJob &J)
{
    if (J.kind != SEED_ROTATED) return J.nlines;
    // the classify pass counts past its capacity; only stored entries exist
    const int64_t cnt = 4 * (int64_t)(*J.rot_count);
    return cnt < J.nlines ? cnt : J.nlines;
}

// Seed position of a line and the S0 normal used for the Eq. step / Eq. tol scaling
// (zero for rotated S0, whose normal is along B). CYL: cylinder jobs may occur (the
// kernels that never see them leave out their trigonometry).
template <bool CYL = true>
__device__ __forceinline__ void seed_of_line(const TraceJob &J, int64_t line, double r[3],
                                             double nrm[3])
{
    nrm[0] = J.normal[0];
    nrm[1] = J.normal[1];
    nrm[2] = J.normal[2];
    if (J.kind == SEED_LIST) {
        const FQ_GLOBAL double *sd = gptr(J.seeds);
        r[0] = sd[3 * line + 0];
        r[1] = sd[3 * line + 1];
        r[2] = sd[3 * line + 2];
    } else if (J.kind == SEED_ROTATED) {
        const FQ_GLOBAL RotEntry &e = gptr(J.rot)[line >> 2];
        const int which = (int)(line & 3);
        const double *d = (which < 2) ? e.U : e.V;
        const double s = (which & 1) ? J.rot_delta : -J.rot_delta;
        for (int a = 0; a < 3; a++) r[a] = e.r0[a] + s * d[a];
        nrm[0] = nrm[1] = nrm[2] = 0.0;
    } else if (CYL && J.kind == SEED_CYL) {
        // a seed on the cylinder; the S0 normal is its outward normal there
        const int64_t i = line % J.dims[0], j = line / J.dims[0];
        const double t = J.s_origin[0] + (double)i * J.s_a[0];
        const double ct = cos(t), st = sin(t);
        r[0] = J.cyl[0] + J.cyl[2] * ct;
        r[1] = J.cyl[1] + J.cyl[2] * st;
        r[2] = J.s_origin[1] + (double)j * J.s_b[1];
        nrm[0] = ct;
        nrm[1] = st;
        nrm[2] = 0.0;
    } else {
        const int64_t i = line % J.dims[0];
        const int64_t j = (line / J.dims[0]) % J.dims[1];
        const int64_t k = line / (J.dims[0] * J.dims[1]);
        for (int a = 0; a < 3; a++)
            r[a] = J.s_origin[a] + (double)i * J.s_a[a] + (double)j * J.s_b[a] +
                   (double)k * J.s_c[a];
    }
}

// Axis a of a job on a stretched grid: the cell holding coordinate r (bisection in
// the node coordinates of a stretched axis, Section 2.2; the floor of the grid
// coordinate on a uniform one) and the local coordinate in it, within [0, 1].
__device__ __forceinline__ int str_cell(const TraceJob &J, int a, double r, double &p)
{
    if (!J.planes.coord[a]) {
        const double g = (r - J.origin[a]) * J.inv_spacing[a];
        const int c = min(max((int)floor(g), 0), J.n[a] - 2);
        p = g - c;
        return c;
    }
    const FQ_GLOBAL double *x = gptr(J.planes.coord[a]);
    const int c = axis_cell((const double *)x, J.n[a], r);
    // a point on the cell's upper node (the box's last node) is at exactly 1
    const double t = r == x[c + 1] ? 1.0 : (r - x[c]) * gptr(J.iw[a])[c];
    p = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    return c;
}

// 1 / the width of cell c along axis a of job J's grid.
__device__ __forceinline__ double inv_width(const TraceJob &J, int a, int c)
{
    return J.iw[a] ? gptr(J.iw[a])[c] : J.inv_spacing[a];
}

// The position along axis a of local coordinate p in cell c of job J's grid.
__device__ __forceinline__ double grid_pos(const TraceJob &J, int a, int c, double p)
{
    const double *x = J.planes.coord[a];
    if (!x) return J.origin[a] + ((double)c + p) * J.spacing[a];
    const FQ_GLOBAL double *xg = gptr(x);
    return xg[c] + p * (xg[c + 1] - xg[c]);
}

// floor(n / d) for 0 <= n < 2^31 with a precomputed 1/d (one FP64 multiply and
// an exact integer correction)
__device__ __forceinline__ int64_t fdiv(int64_t n, int64_t d, double inv_d, int64_t &rem)
{
    int64_t q = (int64_t)((double)n * inv_d);
    int64_t r = n - q * d;
    if (r < 0) {
        q--;
        r += d;
    } else if (r >= d) {
        q++;
        r -= d;
    }
    rem = r;
    return q;
}

// Line of queue item t of a job; -1 for tile holes. Plane seeds come in 8x8 tiles,
// voxels in 4x4x4 tiles (64 neighbouring seeds per wave), lists in order. Tiles are
// taken in the job's tile order when it has one.
__device__ __forceinline__ int64_t line_of_item(const TraceJob &J, int64_t t)
{
    if (J.kind == SEED_LIST || J.kind == SEED_ROTATED) return t < live_lines(J) ? t : -1;
    int64_t ti = t >> 6;
    if (J.tile_order) ti = gptr(J.tile_order)[ti];
    const int w = (int)(t & 63);
    int64_t r0, i, j, k;
    const int64_t q0 = fdiv(ti, J.tiles[0], J.inv_t0, r0);
    if (J.kind == SEED_PLANE || J.kind == SEED_CYL) {
        i = r0 * 8 + (w & 7);
        j = q0 * 8 + (w >> 3);
        k = 0;
    } else {
        int64_t r1;
        const int64_t q1 = fdiv(q0, J.tiles[1], J.inv_t1, r1);
        i = r0 * 4 + (w & 3);
        j = r1 * 4 + ((w >> 2) & 3);
        k = q1 * 4 + (w >> 4);
    }
    if (i >= J.dims[0] || j >= J.dims[1] || k >= J.dims[2]) return -1;
    return (k * J.dims[1] + j) * J.dims[0] + i;
}

}  // namespace dev
}  // namespace fq
