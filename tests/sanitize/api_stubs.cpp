// Host-only stand-ins for the library's kernel launchers, so that the C-ABI layer
// (argument checks, workspace carving, launch sequencing in api.cpp) can run on a
// machine without a GPU under AddressSanitizer and UBSan. Every stub checks that the
// workspace ranges it is handed lie inside the caller's workspace, and counts calls.
#include <stdio.h>
#include <stdlib.h>

#include "fq_internal.h"

namespace fq {

const char *g_ws_lo = nullptr;
const char *g_ws_hi = nullptr;
long g_calls = 0;

static void in_ws(const void *p, size_t bytes, const char *what)
{
    const char *c = (const char *)p;
    if (!g_ws_lo || c < g_ws_lo || c + bytes > g_ws_hi) {
        fprintf(stderr, "%s: [%p, +%zu) outside the workspace [%p, %p)\n", what, p, bytes,
                (const void *)g_ws_lo, (const void *)g_ws_hi);
        abort();
    }
}

hipError_t launch_prep(const fq_field &f, int prec, int want_tw, void *nodes, float *bmax2, hipStream_t)
{
    const size_t n = (size_t)(f.n[0] * f.n[1] * f.n[2]);
    in_ws(nodes, n * (want_tw ? 8 : 4) * (prec == FQ_PREC_F64 ? 8 : 4), "prep nodes");
    in_ws(bmax2, sizeof(float), "prep bmax");
    g_calls++;
    return hipSuccess;
}
hipError_t launch_geometry(const fq_field &f, double *const iw[3], Geo *geo, hipStream_t)
{
    for (int a = 0; a < 3; a++) in_ws(iw[a], (size_t)(f.n[a] - 1) * sizeof(double), "geometry widths");
    in_ws(geo, sizeof(Geo), "geometry record");
    g_calls++;
    return hipSuccess;
}
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t, hipStream_t)
{
    in_ws(p, (size_t)n * 4, "fill");
    g_calls++;
    return hipSuccess;
}
hipError_t launch_store_job(const TraceJob &j, TraceJob *dst, hipStream_t)
{
    in_ws(dst, sizeof *dst, "job table");
    in_ws(j.rec.st, (size_t)(2 * j.nlines) * 2, "half-line status records");
    in_ws(j.rec.end, (size_t)(2 * j.nlines) * 24, "half-line end records");
    g_calls++;
    return hipSuccess;
}
hipError_t launch_trace(int, int, int, const TraceJob *jobs, const TraceParams &tp,
                        unsigned long long *counter, int, int, hipStream_t)
{
    in_ws(jobs, (size_t)tp.njobs * sizeof(TraceJob), "trace jobs");
    in_ws(counter, 8, "trace counter");
    if (tp.list) in_ws(tp.list, (size_t)tp.list_cap * sizeof(FixEntry), "re-trace list");
    if (tp.tape) in_ws(tp.tape, (size_t)tp.pool_cap * sizeof(Ckpt), "checkpoint pool");
    if (tp.tape && tp.list) {
        // the adjoint keeps the checkpoints of the first pass only (the kernels refuse
        // a taped re-trace list)
        fprintf(stderr, "a re-trace pass was launched with the checkpoint pool\n");
        abort();
    }
    g_calls++;
    return hipSuccess;
}
hipError_t launch_bucket_order(int64_t n, int32_t *key, uint32_t *counts, int32_t *order, hipStream_t)
{
    in_ws(key, (size_t)n * 4, "bucket keys");
    in_ws(counts, 256 * 4, "bucket counts");
    in_ws(order, (size_t)n * 4, "bucket order");
    g_calls++;
    return hipSuccess;
}
hipError_t launch_tile_order(const TraceJob &J, int, int, int32_t *bucket, uint32_t *counts,
                             int32_t *order, hipStream_t s)
{
    return launch_bucket_order(J.tiles[0] * J.tiles[1], bucket, counts, order, s);
}
hipError_t launch_voxel_order(const TraceJob &J, int, int, int32_t *key, uint32_t *counts,
                              int32_t *order, hipStream_t)
{
    const size_t n = (size_t)(J.tiles[0] * J.tiles[1] * J.tiles[2]);
    in_ws(key, n * 4, "voxel tile keys");
    in_ws(counts, 65536 * 4, "voxel key counts");
    in_ws(order, n * 4, "voxel tile order");
    g_calls++;
    return hipSuccess;
}
hipError_t launch_graze(const TraceJob *jobs, int job, int64_t, double, const double *, double,
                        FixEntry *list, uint32_t *count, uint32_t *count_tw, int64_t cap, int, int,
                        hipStream_t)
{
    in_ws(jobs + job, sizeof(TraceJob), "graze job");
    in_ws(list, (size_t)cap * sizeof(FixEntry), "graze list");
    in_ws(count, 4, "graze count");
    in_ws(count_tw, 4, "graze twist count");
    g_calls++;
    return hipSuccess;
}
hipError_t launch_fix_order(const TraceJob *, const FixEntry *list, const uint32_t *count, int64_t cap,
                            int32_t *key, uint32_t *counts, FixEntry *out, hipStream_t)
{
    in_ws(list, (size_t)cap * sizeof(FixEntry), "re-trace list");
    in_ws(count, 4, "re-trace count");
    in_ws(key, (size_t)cap * 4, "re-trace keys");
    in_ws(counts, 256 * 4, "re-trace key counts");
    in_ws(out, (size_t)cap * sizeof(FixEntry), "ordered re-trace list");
    g_calls++;
    return hipSuccess;
}
hipError_t launch_map_backward(const MapJob &m, const double *, const double *, const double *,
                               const double *, double *lam_end, double *lam_tw, double *gnode,
                               int64_t nhalf0, hipStream_t)
{
    const size_t halves = (size_t)(nhalf0 + (m.rot_index ? 2 * m.rot_nlines : 0));
    in_ws(lam_end, halves * 24, "end adjoints");
    in_ws(lam_tw, halves * 8, "twist adjoints");
    in_ws(gnode, (size_t)(m.n[0] * m.n[1] * m.n[2]) * 24, "node gradients");
    g_calls++;
    return hipSuccess;
}
hipError_t launch_rot_seed(const MapJob &m, const RotEntry *rot, const uint32_t *rot_count, int64_t cap,
                           const double *lam_seed, double *gnode, hipStream_t)
{
    in_ws(rot, (size_t)cap * sizeof(RotEntry), "rotated-S0 entries");
    in_ws(rot_count, 4, "rotated-S0 count");
    in_ws(lam_seed, (size_t)(2 * m.rot_nlines) * 24, "seed adjoints");
    in_ws(gnode, (size_t)(m.n[0] * m.n[1] * m.n[2]) * 24, "node gradients");
    g_calls++;
    return hipSuccess;
}
hipError_t launch_bwd_order(const int32_t *acc, int64_t nh, int32_t *key, uint32_t *counts,
                            int32_t *order, hipStream_t s)
{
    in_ws(acc, (size_t)nh * 4, "accepted steps per half");
    return launch_bucket_order(nh, key, counts, order, s);
}
hipError_t launch_trace_backward(int, int, const TraceJob *job, const BwdParams &bp, hipStream_t)
{
    in_ws(job, sizeof(TraceJob), "reverse job");
    in_ws(bp.buf, (size_t)bp.nslots * bp.seg * sizeof(StepRec), "replay buffers");
    in_ws(bp.order, (size_t)bp.nhalves * 4, "reverse order");
    g_calls++;
    return hipSuccess;
}
hipError_t launch_grad_planes(const fq_field &, const double *gnode, int, double *const gb[3], hipStream_t)
{
    in_ws(gnode, 8, "node gradients");
    if (!gb[0] || !gb[1] || !gb[2]) abort();
    g_calls++;
    return hipSuccess;
}
hipError_t launch_classify(const MapJob &m, int32_t *rot_index, RotEntry *rot, uint32_t *rot_count,
                           int64_t cap, hipStream_t)
{
    in_ws(rot_index, (size_t)m.nlines * 4, "rotated index");
    in_ws(rot, (size_t)cap * sizeof(RotEntry), "rotated list");
    in_ws(rot_count, 4, "rotated count");
    in_ws(m.rot_rec.st, (size_t)(2 * m.rot_nlines) * 2, "rotated records");
    g_calls++;
    return hipSuccess;
}
hipError_t launch_stencil(const MapJob &m, hipStream_t)
{
    in_ws(m.rec.st, (size_t)(2 * m.nlines) * 2, "stencil records");
    g_calls++;
    return hipSuccess;
}
hipError_t launch_m2_map(const MapJob &m, hipStream_t)
{
    in_ws(m.rec.st, (size_t)(2 * m.nlines) * 2, "Method II records");
    in_ws(m.rec.uv, (size_t)(2 * m.nlines) * 48, "Method II tangent vectors");
    g_calls++;
    return hipSuccess;
}
hipError_t launch_rot_ranges(TraceJob *jobs, int first, int n, int64_t, int64_t *total, hipStream_t)
{
    in_ws(jobs + first, (size_t)n * sizeof(TraceJob), "rotated jobs");
    in_ws(total, sizeof(int64_t), "queue total");
    g_calls++;
    return hipSuccess;
}
hipError_t launch_cyl_map(const MapJob &m, hipStream_t)
{
    in_ws(m.rec.end, (size_t)(2 * m.nlines) * 24, "line records");
    g_calls++;
    return hipSuccess;
}
hipError_t launch_perp_map(const MapJob &m, int, hipStream_t)
{
    in_ws(m.rec.end, (size_t)(2 * m.nlines) * 24, "line records");
    g_calls++;
    return hipSuccess;
}
hipError_t launch_lines_out(const MapJob &m, const double *, hipStream_t)
{
    in_ws(m.rec.end, (size_t)(2 * m.nlines) * 24, "line records");
    g_calls++;
    return hipSuccess;
}

}  // namespace fq

// The HIP runtime calls of the host layer: events and the error state, without a GPU.
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
