// Internal definitions shared by the library's translation units (host + device).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fastqsl.h"
#include "field64.h"

namespace fq {

// How a trace job enumerates its seeds.
enum SeedKind : int32_t {
    SEED_LIST = 0,    // explicit device array of n x 3 doubles
    SEED_PLANE = 1,   // origin + i a + j b   (a = du u, b = dv v)
    SEED_VOXELS = 2,  // origin + i a + j b + k c (a, b, c along the axes)
    SEED_ROTATED = 3, // r0 +- delta U, r0 +- delta V of the rotated-S0 list
    SEED_CYL = 4,     // (xc + R cos(t0 + i dt), yc + R sin(t0 + i dt), z0 + j dz)
};

// face id of a half line that ends on a cylindrical mapping surface
constexpr int kFaceCyl = FQ_FACE_CYL;

// One rotated-S0 point: its map index, centre and in-plane unit vectors.
struct RotEntry {
    int64_t point;
    double r0[3];
    double U[3];
    double V[3];
};

// Half-line records written by the tracer. Half 0 runs against B (backward),
// half 1 along it (forward); record (half, line) is at half * nlines + line.
struct HalfRecs {
    double *end;   // 2 * nlines * 3
    double *tw;    // 2 * nlines
    double *len;   // 2 * nlines
    int8_t *face;  // 2 * nlines
    uint16_t *st;  // 2 * nlines
    double *uv;    // Method II: 2 * nlines * 6, the tangent vectors U, V at the end (else NULL)
};

// Stretched grids: what the geometry pass finds on the device.
struct Geo {
    double dref;   // smallest cell width over the three axes (the tracer's length unit)
    int32_t bad;   // nonzero: node coordinates not strictly increasing and finite, or not
                   // spanning the box that origin and spacing give
    int32_t pad;
};

// One independent tracing job: a prepared field plus a seed set.
struct TraceJob {
    const void *nodes;   // node records in the compute type: (Bx, By, Bz, Jx, Jy, Jz, 0, 0)
                         // with the twist integrand, else (Bx, By, Bz, 0)
    const float *bmax2;  // max |B|^2 over the nodes (float, written by the prep pass)
    int32_t n[3];
    int32_t kind;
    double origin[3];
    double spacing[3];
    // seeds
    int32_t tile[3];     // seeds per tile along each seed axis (tile volume <= 64)
    int32_t pad;
    int64_t dims[3];     // seed grid extents (list: n,1,1; rotated: 4*capacity,1,1)
    int64_t tiles[3];    // tiles along each seed axis
    int64_t nitems;      // queue items per half = tiles volume * tile volume
    int64_t nlines;      // output lines of the job
    double s_origin[3];
    double s_a[3], s_b[3], s_c[3];
    double normal[3];    // S0 normal (Eq. step / Eq. tol scaling)
    double cyl[3];       // SEED_CYL: axis (xc, yc) and radius R; seeds use s_origin[0] = t0,
                         // s_a[0] = dt, s_origin[1] = z0, s_b[1] = dz; lines run inside it
    const double *seeds;          // SEED_LIST
    const RotEntry *rot;          // SEED_ROTATED
    const uint32_t *rot_count;    // SEED_ROTATED: number of valid entries
    double rot_delta;             // SEED_ROTATED: distance of the extra seeds
    HalfRecs rec;
    int64_t item_base;   // first queue item of the job (items of both halves follow)
    const int32_t *tile_order;  // plane jobs: tiles in the order they are traced (may be NULL)
    Planes64 planes;     // the caller's field, for FP64 angles in the grazing test
    // stretched grids (NULL on a uniform grid): per-cell 1 / width of every axis (a
    // uniform axis repeats 1 / spacing) and the grid's reference length; the node
    // coordinates of the stretched axes themselves are in planes.coord
    const double *iw[3];
    const Geo *geo;
    // precomputed per-job constants of the tracer
    float rscale[3];     // reference length / spacing per axis (uniform grids)
    float twk;           // reference length / (4 pi) (uniform grids)
    double dref;         // reference length (smallest spacing; uniform grids)
    double inv_spacing[3];
    double inv_t0, inv_t1; // 1 / tiles[0], 1 / tiles[1] (tile decode)
};

// One half line to trace again (FP64 pass).
struct FixEntry {
    int32_t job;
    int32_t half;  // 0 backward, 1 forward
    int64_t line;
};

// Lane state at a checkpoint of the adjoint's forward pass (64 bytes): enough to
// replay the half line from there exactly. Checkpoints come from one pool; those of
// a half line are chained from its last one backwards.
struct Ckpt {
    double p0, p1, p2, h, tol;
    int32_t c0, c1, c2, force;
    int32_t trials;
    int32_t prev;  // pool slot of the previous checkpoint of the half line, -1 = none
};

// One accepted step found by a replay, for the reverse sweep (56 bytes).
struct StepRec {
    double p0, p1, p2;  // local position before the step
    double H;           // step length in the independent variable
    int32_t c0, c1, c2;
    int32_t axis;       // landing axis, -1 for a plain step
    int32_t clamp;      // bit q: coordinate q was clamped onto a box face
    int32_t pad;
};

struct TraceParams {
    double tol_perp, step_perp, step_min, tol_floor;
    int64_t max_steps;
    int32_t want_tw;
    int32_t njobs;
    int64_t static_items;          // queue items of the main jobs (before the rotated ones)
    int32_t dynamic_last;          // 1 if rotated-S0 jobs follow the main jobs: their item
                                   // ranges and the queue's size (*total_dev) are set on
                                   // the device once the classify passes have counted them
    const int64_t *total_dev;
    int32_t cyl;                   // some job runs inside a cylindrical mapping surface
                                   // (multi-job kernels then)
    unsigned long long *stats;     // optional counters (trials, accepted, fetches, halves, FP64 halves)
    const FixEntry *list;          // list mode: trace exactly these half lines
    const uint32_t *list_count;
    int64_t list_cap;
    int32_t list_rev;              // list mode: entry k sits at list[list_cap - 1 - k]
    int32_t scheme;                // integration scheme (FQ_SCHEME_*)
    int32_t method;                // FQ_METHOD_I or FQ_METHOD_II (tangent vectors carried)
    int32_t stretched;             // some job's grid is stretched (multi-job kernels then)
    // adjoint forward pass (FP64, single job): checkpoints every `seg` accepted steps
    Ckpt *tape;                    // checkpoint pool of pool_cap entries
    unsigned long long *pool_ctr;  // next free pool slot
    int32_t *tape_last;            // per half record: pool slot of its last checkpoint
    int32_t *tape_n;               // per half record: checkpoints stored
    int32_t *tape_acc;             // per half record: accepted steps
    int32_t seg;
    int32_t pad2;
    int64_t pool_cap;
    int64_t tape_base1;            // first record of job 1 (a rotated-S0 job) in tape_*
    // per-XCD queues (multi-job kernels, not list mode): when set, 8 counters 64 bytes
    // apart, one per range of the queue split in 8 contiguous ranges of whole tiles
    unsigned long long *xcd_ctr;
};

// Reverse sweep over the traced half lines of one job.
struct BwdParams {
    const Ckpt *tape;
    const int32_t *tape_last, *tape_n, *tape_acc;
    int32_t seg, pad0;
    int64_t nhalves;               // 2 * nlines
    const double *lam_end;         // per half: dL/d(end point), 3 doubles
    const double *lam_tw;          // per half: dL/d(Tw of the half)
    double *gnode;                 // 6 planes over the nodes: dL/d(Bx, By, Bz, Jx, Jy, Jz)
    StepRec *buf;                  // nslots * seg replay records
    int64_t nslots;                // lanes of the reverse kernel
    unsigned long long *counter;   // queue
    const int32_t *order;          // the half lines in queue order (longest first)
    unsigned long long *stats;     // optional: halves, steps, replay mismatches, dropped halves
    int64_t max_steps;
    int32_t want_tw;
    int32_t scheme;                // Scheme of the forward pass (trace_core.h)
    // an interior seed plane: jobs[1] is its rotated-S0 job, whose half lines follow
    // the plane's nhalf0 ones; the adjoint at each of their seeds goes to lam_seed
    // (3 per half of the rotated job, physical units)
    int64_t nhalf0;
    double *lam_seed;
};

// Host-side launchers, one per translation unit.
hipError_t launch_prep(const fq_field &f, int prec, int want_tw, void *nodes, float *bmax2,
                       hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
// The queue ranges of the rotated-S0 jobs jobs_dev[first .. first + n): items from
// `base` on, each job's item count its live lines rounded up to a wave, both halves;
// the queue's end goes to *total.
hipError_t launch_rot_ranges(TraceJob *jobs_dev, int first, int n, int64_t base, int64_t *total,
                             hipStream_t s);
// Stretched grids: the geometry pass (per-cell 1 / width of all three axes into
// iw[a][0 .. n[a]-2], and *geo).
struct GeoIn {
    const double *coord[3];
    int32_t n[3];
    int32_t pad;
    double spacing[3];
    double origin[3];
};
hipError_t launch_geometry(const fq_field &f, double *const iw[3], Geo *geo, hipStream_t s);
hipError_t launch_store_job(const TraceJob &j, TraceJob *dst, hipStream_t s);
// prec: compute type (FQ_PREC_F32X = float, FQ_PREC_F64 = double);
// store: node-record type (FQ_DT_F32 / FQ_DT_F64);
// twm: 0 = no twist, 1 = twist, 2 = positions only on twist-layout records, keeping the
// twist already in the records (the FP64 re-trace); 3 = as 2 at three waves per SIMD
// (FP64 only: for calls that share the GPU with other maps in flight).
hipError_t launch_trace(int prec, int store, int twm, const TraceJob *jobs_dev,
                        const TraceParams &tp, unsigned long long *counter, int block,
                        int waves_per_cu, hipStream_t s);
// Order n items longest first: key (n values, 0..255 = longest; overwritten with the
// bucket), counts (256), order (n: the item indices in queue order) are workspace.
hipError_t launch_bucket_order(int64_t n, int32_t *key, uint32_t *counts, int32_t *order,
                               hipStream_t s);
// Order the tiles of a plane job (J: its host copy; its node records, written by
// the prep pass for precision prec and want_tw, valid on the device): bucket (tiles),
// counts (256), order (tiles) are workspace arrays.
hipError_t launch_tile_order(const TraceJob &J, int prec, int want_tw, int32_t *bucket, uint32_t *counts,
                             int32_t *order, hipStream_t s);
hipError_t launch_voxel_order(const TraceJob &J, int prec, int want_tw, int32_t *key,
                              uint32_t *counts, int32_t *order, hipStream_t s);
// Lists the half lines of job `job` that the FP64 pass traces again at
// list[0, *count) and, with split, the half lines the FP32 pass could not finish
// (whose twist is then missing too) apart at list[cap - 1 - k] for k < *count_tw.
// qmap: the job's map after the FP32 pass (the map of the job's main points for a
// rotated-S0 job), or NULL. seed_check: also list lines whose seed is grazing.
// The first `*count` entries of the FP64 pass's list, longest half lines first, into
// `out` (key: cap int32, counts: 256 uint32 of scratch).
hipError_t launch_fix_order(const TraceJob *jobs_dev, const FixEntry *list, const uint32_t *count,
                            int64_t cap, int32_t *key, uint32_t *counts, FixEntry *out,
                            hipStream_t s);
hipError_t launch_graze(const TraceJob *jobs_dev, int job, int64_t max_lines, double thr,
                        const double *qmap, double qthr, FixEntry *list, uint32_t *count,
                        uint32_t *count_tw, int64_t cap, int split, int seed_check, hipStream_t s);

// Map assembly (Q stencil) of one layer-structured map.
struct MapJob {
    const void *b[3];     // input planes (original dtype) for FP64 B_n
    int32_t dtype;
    int32_t n[3];
    double origin[3], spacing[3];
    const double *coord[3];  // node coordinates of stretched axes (NULL = uniform axis)
    int64_t nu, nv, nlayers;     // points per layer = nu*nv
    double d0, d1;               // seed spacing along the two S0 axes
    double normal[3];            // S0 normal
    double p_origin[3], p_a[3], p_b[3], p_c[3]; // point(i,j,k) = origin + i a + j b + k c
    int32_t on_face;             // every seed lies on a box face (no rotation)
    int32_t is_cyl;              // a cylinder map: points (theta, z), S0 = S1 = S2 = the cylinder
    double cyl[3];               // its axis (xc, yc) and radius
    double edge_eps;
    HalfRecs rec;                // records of the map's own lines (nlines = points)
    int64_t nlines;
    const int32_t *rot_index;    // per point: index in the rotated list or -1 (may be NULL)
    const RotEntry *rot;
    HalfRecs rot_rec;            // records of the rotated extras (4 per entry)
    int64_t rot_nlines;
    double rot_delta;
    fq_map out;
};

// Adjoint (adjoint.hip).
hipError_t launch_map_backward(const MapJob &m, const double *dq, const double *dtw,
                               const double *dend_b, const double *dend_f, double *lam_end,
                               double *lam_tw, double *gnode, int64_t nhalf0, hipStream_t s);
hipError_t launch_rot_seed(const MapJob &m, const RotEntry *rot, const uint32_t *rot_count,
                           int64_t cap, const double *lam_seed, double *gnode, hipStream_t s);
// Queue order of the reverse kernel: half lines by their accepted steps, most first
// (key, counts, order: workspace of nhalves, 256 and nhalves entries).
hipError_t launch_bwd_order(const int32_t *tape_acc, int64_t nhalves, int32_t *key,
                            uint32_t *counts, int32_t *order, hipStream_t s);
hipError_t launch_trace_backward(int store, int want_tw, const TraceJob *job_dev,
                                 const BwdParams &bp, hipStream_t s);
hipError_t launch_grad_planes(const fq_field &f, const double *gnode, int want_tw,
                              double *const gb[3], hipStream_t s);
constexpr int64_t kBwdSlots = 32768;  // lanes of the reverse kernel

hipError_t launch_classify(const MapJob &m, int32_t *rot_index, RotEntry *rot,
                           uint32_t *rot_count, int64_t rot_capacity, hipStream_t s);
hipError_t launch_stencil(const MapJob &m, hipStream_t s);
// Method II: Q and Q_perp of every point from its own line's tangent vectors.
hipError_t launch_m2_map(const MapJob &m, hipStream_t s);
// Method I Q_perp (S1, S2 perpendicular to B at the ends; want_qperp) and the length
// edge map |grad_S0 length| of a map, from its lines' records and stencil.
hipError_t launch_perp_map(const MapJob &m, int want_qperp, hipStream_t s);
// Method I Q of a cylinder map (surface coordinates on the cylinder).
hipError_t launch_cyl_map(const MapJob &m, hipStream_t s);
hipError_t launch_lines_out(const MapJob &m, const double *seeds_list, hipStream_t s);

}  // namespace fq
