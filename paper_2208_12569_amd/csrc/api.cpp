// C-ABI entry points: argument checks, workspace carving and launch sequencing.
//
// Every call enqueues, on the caller's stream and into the caller's workspace:
//   fill (counters)  ->  prep (node records + curl, per field)
//   -> [classify (rotated-S0 list)] -> store job table -> persistent trace
//   -> stencil (Q, Tw, length, per-line outputs)
// The size query and the call carve the workspace with the same code path, so the
// two can never disagree.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "fq_internal.h"

namespace fq {
namespace {

struct Carve {
    size_t off = 0;
    size_t take(size_t bytes)
    {
        size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    }
};

enum SpecKind { SPEC_LIST, SPEC_PLANE, SPEC_VOXELS, SPEC_CYL };

struct Spec {
    SpecKind kind;
    const fq_field *f;
    fq_plane pl;
    fq_voxels vx;
    fq_cylinder cy;
    const double *seeds;
    int64_t nlist;
    double normal[3];
    const fq_map *map;        // maps (plane / voxels)
    const fq_lines *lines;    // list outputs
};

int64_t nodes_of(const fq_field *f) { return f->n[0] * f->n[1] * f->n[2]; }

bool stretched(const fq_field *f) { return f->coord[0] || f->coord[1] || f->coord[2]; }

int64_t lines_of(const Spec &s)
{
    switch (s.kind) {
    case SPEC_LIST: return s.nlist;
    case SPEC_PLANE: return s.pl.nu * s.pl.nv;
    case SPEC_CYL: return s.cy.ntheta * s.cy.nz;
    default: return s.vx.n[0] * s.vx.n[1] * s.vx.n[2];
    }
}

bool finite3(const double v[3]) { return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]); }

int check_field(const fq_field *f)
{
    if (!f) return FQ_EINVAL;
    for (int a = 0; a < 3; a++) {
        if (f->n[a] < 2 || f->n[a] > 65535) return FQ_EINVAL;  // grid extents of the prep pass
        if (!f->b[a]) return FQ_EINVAL;
        // on a stretched axis these give the box extent (the geometry pass checks them
        // against the node coordinates)
        if (!(f->spacing[a] > 0.0) || !isfinite(f->spacing[a])) return FQ_EINVAL;
        if (!isfinite(f->origin[a])) return FQ_EINVAL;
    }
    if (f->dtype != FQ_DT_F32 && f->dtype != FQ_DT_F64) return FQ_EINVAL;
    if (nodes_of(f) > ((int64_t)1 << 40)) return FQ_EINVAL;
    return FQ_OK;
}

int check_plane(const fq_plane *p)
{
    if (!p) return FQ_EINVAL;
    if (p->nu < 1 || p->nv < 1 || (p->nu * p->nv) > ((int64_t)1 << 34)) return FQ_EINVAL;
    if (!(p->du > 0.0) || !(p->dv > 0.0) || !isfinite(p->du) || !isfinite(p->dv)) return FQ_EINVAL;
    if (!finite3(p->origin) || !finite3(p->u) || !finite3(p->v)) return FQ_EINVAL;
    double uu = p->u[0] * p->u[0] + p->u[1] * p->u[1] + p->u[2] * p->u[2];
    double vv = p->v[0] * p->v[0] + p->v[1] * p->v[1] + p->v[2] * p->v[2];
    double uv = p->u[0] * p->v[0] + p->u[1] * p->v[1] + p->u[2] * p->v[2];
    if (fabs(uu - 1.0) > 1e-9 || fabs(vv - 1.0) > 1e-9 || fabs(uv) > 1e-9) return FQ_EINVAL;
    return FQ_OK;
}

// A cylinder map: points, radius, steps; the cylinder inside the box in x and y.
int check_cylinder(const fq_cylinder *c, const fq_field *f)
{
    if (!c) return FQ_EINVAL;
    if (c->ntheta < 1 || c->nz < 1 || c->ntheta * c->nz > ((int64_t)1 << 34)) return FQ_EINVAL;
    if (!(c->radius > 0.0) || !isfinite(c->radius)) return FQ_EINVAL;
    if (!isfinite(c->theta0) || !isfinite(c->dtheta) || !isfinite(c->z0) || !isfinite(c->dz) ||
        !isfinite(c->centre[0]) || !isfinite(c->centre[1]))
        return FQ_EINVAL;
    for (int a = 0; a < 2; a++) {
        const double lo = f->origin[a], hi = f->origin[a] + (f->n[a] - 1) * f->spacing[a];
        if (!(c->centre[a] - c->radius >= lo && c->centre[a] + c->radius <= hi)) return FQ_EINVAL;
    }
    return FQ_OK;
}

int check_voxels(const fq_voxels *v)
{
    if (!v) return FQ_EINVAL;
    for (int a = 0; a < 3; a++) {
        if (v->n[a] < 1) return FQ_EINVAL;
        if (!(v->spacing[a] > 0.0) || !isfinite(v->spacing[a])) return FQ_EINVAL;
    }
    if (v->n[0] * v->n[1] * v->n[2] > ((int64_t)1 << 34)) return FQ_EINVAL;
    if (!finite3(v->origin)) return FQ_EINVAL;
    return FQ_OK;
}

// Default error-bound floors (grid spacings): 16 ulp(1) of FP32 and about 70 ulp(1)
// of FP64.
constexpr double kFloor32 = 2.384185791015625e-7, kFloor64 = 1e-14;

int resolve_params(const fq_params *in, fq_params &p)
{
    memset(&p, 0, sizeof p);
    if (in) p = *in;
    if (p.precision != FQ_PREC_F32X && p.precision != FQ_PREC_F64) return FQ_EINVAL;
    if (p.tol_perp < 0 || p.step_perp < 0 || p.step_min < 0 || p.tol_floor < 0 || p.edge_eps < 0 ||
        p.max_steps < 0)
        return FQ_EINVAL;
    if (!isfinite(p.tol_perp) || !isfinite(p.step_perp) || !isfinite(p.step_min) ||
        !isfinite(p.tol_floor) || !isfinite(p.edge_eps))
        return FQ_EINVAL;
    if (p.block != 0 && (p.block < 64 || p.block > 256 || (p.block % 64) != 0)) return FQ_EINVAL;
    if (p.waves_per_cu < 0) return FQ_EINVAL;
    if (p.tol_perp == 0) p.tol_perp = 1e-6;
    if (p.step_perp == 0) p.step_perp = 1.0;
    if (p.step_min == 0) p.step_min = 0.05;
    if (p.tol_floor == 0) p.tol_floor = (p.precision == FQ_PREC_F64) ? kFloor64 : kFloor32;
    if (p.edge_eps == 0) p.edge_eps = 1e-5;
    if (p.max_steps == 0) p.max_steps = 200000;
    if (!isfinite(p.graze)) return FQ_EINVAL;
    if (p.graze == 0) p.graze = 0.05;
    if (!isfinite(p.qfix)) return FQ_EINVAL;
    if (p.qfix == 0) p.qfix = 300.0;
    if (p.scheme < FQ_SCHEME_RKF45 || p.scheme > FQ_SCHEME_RK4_38) return FQ_EINVAL;
    if (p.method != FQ_METHOD_I && p.method != FQ_METHOD_II) return FQ_EINVAL;
    if (p.reserved2 != 0) return FQ_EINVAL;
    p.in_flight = p.in_flight != 0;
    if (p.tape_steps < 0) return FQ_EINVAL;
    if (p.tape_steps == 0) p.tape_steps = 2048;
    if (in == nullptr) p.want_tw = 1;
    return FQ_OK;
}

// All seeds of the plane on one box face (then S0 is never rotated).
bool plane_on_face(const fq_plane &pl, const fq_field &f)
{
    double n[3] = {pl.u[1] * pl.v[2] - pl.u[2] * pl.v[1], pl.u[2] * pl.v[0] - pl.u[0] * pl.v[2],
                   pl.u[0] * pl.v[1] - pl.u[1] * pl.v[0]};
    for (int a = 0; a < 3; a++) {
        if (fabs(fabs(n[a]) - 1.0) > 1e-12) continue;
        double lo = f.origin[a], hi = f.origin[a] + (f.n[a] - 1) * f.spacing[a];
        double tol = 1e-12 * f.spacing[a];
        if (fabs(pl.origin[a] - lo) <= tol || fabs(pl.origin[a] - hi) <= tol) return true;
    }
    return false;
}

struct SpecWs {
    size_t nodes, bmax, end, tw, len, face, st;
    size_t uv;  // Method II: tangent vectors at the half lines' ends
    size_t iw[3], geo;  // stretched grids: per-cell 1 / width per axis, and the Geo record
    size_t tile_order, tile_bucket, tile_counts;  // plane jobs
    size_t nodes64;  // FP64 node records for the FP64 pass (FP64 grids only)
    size_t rot_index, rot, rot_count, r_end, r_tw, r_len, r_face, r_st;
    bool rotate;
    int64_t nlines;
};

HalfRecs recs_at(char *ws, size_t end, size_t tw, size_t len, size_t face, size_t st)
{
    HalfRecs r;
    r.end = (double *)(ws + end);
    r.tw = (double *)(ws + tw);
    r.len = (double *)(ws + len);
    r.face = (int8_t *)(ws + face);
    r.st = (uint16_t *)(ws + st);
    r.uv = nullptr;
    return r;
}

void take_recs(Carve &cv, int64_t n, size_t &end, size_t &tw, size_t &len, size_t &face, size_t &st)
{
    end = cv.take((size_t)(2 * n) * 3 * sizeof(double));
    tw = cv.take((size_t)(2 * n) * sizeof(double));
    len = cv.take((size_t)(2 * n) * sizeof(double));
    face = cv.take((size_t)(2 * n));
    st = cv.take((size_t)(2 * n) * sizeof(uint16_t));
}

void set_map_geometry(const Spec &s, MapJob &m)
{
    const fq_field &f = *s.f;
    for (int a = 0; a < 3; a++) {
        m.b[a] = f.b[a];
        m.n[a] = (int32_t)f.n[a];
        m.origin[a] = f.origin[a];
        m.spacing[a] = f.spacing[a];
        m.coord[a] = f.coord[a];
    }
    m.dtype = f.dtype;
    if (s.kind == SPEC_PLANE) {
        m.nu = s.pl.nu;
        m.nv = s.pl.nv;
        m.nlayers = 1;
        m.d0 = s.pl.du;
        m.d1 = s.pl.dv;
        for (int a = 0; a < 3; a++) {
            m.p_origin[a] = s.pl.origin[a];
            m.p_a[a] = s.pl.du * s.pl.u[a];
            m.p_b[a] = s.pl.dv * s.pl.v[a];
            m.p_c[a] = 0.0;
            m.normal[a] = s.normal[a];
        }
    } else if (s.kind == SPEC_VOXELS) {
        m.nu = s.vx.n[0];
        m.nv = s.vx.n[1];
        m.nlayers = s.vx.n[2];
        m.d0 = s.vx.spacing[0];
        m.d1 = s.vx.spacing[1];
        for (int a = 0; a < 3; a++) {
            m.p_origin[a] = s.vx.origin[a];
            m.p_a[a] = a == 0 ? s.vx.spacing[0] : 0.0;
            m.p_b[a] = a == 1 ? s.vx.spacing[1] : 0.0;
            m.p_c[a] = a == 2 ? s.vx.spacing[2] : 0.0;
            m.normal[a] = s.normal[a];
        }
    } else if (s.kind == SPEC_CYL) {
        // points (theta, z): theta0 + i dtheta, z0 + j dz on the cylinder
        m.nu = s.cy.ntheta;
        m.nv = s.cy.nz;
        m.nlayers = 1;
        m.d0 = s.cy.radius * s.cy.dtheta;
        m.d1 = s.cy.dz;
        m.is_cyl = 1;
        m.cyl[0] = s.cy.centre[0];
        m.cyl[1] = s.cy.centre[1];
        m.cyl[2] = s.cy.radius;
        m.p_origin[0] = s.cy.theta0;
        m.p_a[0] = s.cy.dtheta;
        m.p_origin[1] = s.cy.z0;
        m.p_b[1] = s.cy.dz;
    } else {
        m.nu = s.nlist;
        m.nv = 1;
        m.nlayers = 1;
        for (int a = 0; a < 3; a++) m.normal[a] = s.normal[a];
    }
}

void set_job_constants(TraceJob &J);

// The reverse-mode call of one q2d map: its output adjoints, the gradient planes and
// the checkpoint layout.
struct BwdSpec {
    // 0: checkpointed forward pass, then the reverse pass (no map written);
    // 1: checkpointed forward pass and the map (a later phase 2 reverses it);
    // 2: the reverse pass of a workspace that phase 1 filled
    int phase;
    int seg;                 // accepted steps between checkpoints
    int64_t pool;            // checkpoints in the pool
    const double *dq, *dtw, *dend_b, *dend_f;
    double *const *gb;
};

// Carve the workspace and (unless dry) enqueue the whole call. With bwd, the trace
// keeps checkpoints and the map is differentiated instead of written, or (phases 1
// and 2) the two halves of that are enqueued by separate calls on one workspace.
int run(const std::vector<Spec> &specs, const fq_params &P, char *ws, size_t ws_bytes, bool dry,
        size_t *need, hipStream_t stream, const BwdSpec *bwd = nullptr)
{
    const int ns = (int)specs.size();
    const size_t tsz = P.precision == FQ_PREC_F64 ? 8 : 4;
    // launches are checked with hipGetLastError: an error that an earlier, unrelated
    // HIP call of the caller left behind is not this call's (a fault still shows, as
    // the sticky error every later call returns)
    if (!dry) (void)hipGetLastError();
    // Method II: maps only (a list of seeds traces plain lines), RKF45, no adjoint
    bool m2 = P.method == FQ_METHOD_II;
    for (int i = 0; i < ns; i++)
        if (specs[i].kind == SPEC_LIST) m2 = false;
    if (m2 && (P.scheme != FQ_SCHEME_RKF45 || bwd)) return FQ_EUNSUPPORTED;
    for (int i = 0; i < ns; i++)
        if (specs[i].kind == SPEC_CYL && (m2 || bwd || P.scheme != FQ_SCHEME_RKF45)) return FQ_EUNSUPPORTED;
    for (int i = 0; i < ns; i++)
        if (stretched(specs[i].f) && m2) return FQ_EUNSUPPORTED;
    Carve cv;
    // queue counters: +0 the tracer (u64, u32 spare), +64 the reverse pass, +128 the
    // checkpoint pool, +192 the FP64 pass over half lines that need their twist
    const size_t off_ctr = cv.take(256);
    // per-XCD queue counters of a 3-D map (8, 64 bytes apart)
    const bool xcd = ns == 1 && specs[0].kind == SPEC_VOXELS;
    const size_t off_xctr = xcd ? cv.take(512) : 0;
    std::vector<SpecWs> W(ns);
    int nrot = 0;
    for (int i = 0; i < ns; i++) {
        const Spec &s = specs[i];
        SpecWs &w = W[i];
        memset(&w, 0, sizeof w);
        const int64_t nn = nodes_of(s.f);
        w.nlines = lines_of(s);
        w.nodes = cv.take((size_t)nn * (P.want_tw ? 8 : 4) * tsz);
        w.bmax = cv.take(sizeof(float));
        take_recs(cv, w.nlines, w.end, w.tw, w.len, w.face, w.st);
        if (s.kind == SPEC_PLANE || s.kind == SPEC_VOXELS) {
            const int64_t ntiles = s.kind == SPEC_PLANE
                                       ? ((s.pl.nu + 7) / 8) * ((s.pl.nv + 7) / 8)
                                       : ((s.vx.n[0] + 3) / 4) * ((s.vx.n[1] + 3) / 4) * ((s.vx.n[2] + 3) / 4);
            w.tile_order = cv.take((size_t)ntiles * sizeof(int32_t));
            w.tile_bucket = cv.take((size_t)ntiles * sizeof(int32_t));
            // voxel tiles are sorted over 65536 footpoint keys, plane tiles over 256
            w.tile_counts = cv.take((s.kind == SPEC_VOXELS ? 65536 : 256) * sizeof(uint32_t));
        }
        if (m2) w.uv = cv.take((size_t)(2 * w.nlines) * 6 * sizeof(double));
        if (stretched(s.f)) {
            for (int a = 0; a < 3; a++) w.iw[a] = cv.take((size_t)(s.f->n[a] - 1) * sizeof(double));
            w.geo = cv.take(sizeof(Geo));
        }
        w.rotate = !m2 && ((s.kind == SPEC_VOXELS) || (s.kind == SPEC_PLANE && !plane_on_face(s.pl, *s.f)));
        if (w.rotate) {
            nrot++;
            w.rot_index = cv.take((size_t)w.nlines * sizeof(int32_t));
            w.rot = cv.take((size_t)w.nlines * sizeof(RotEntry));
            w.rot_count = cv.take(sizeof(uint32_t));
            take_recs(cv, 4 * w.nlines, w.r_end, w.r_tw, w.r_len, w.r_face, w.r_st);
        }
    }
    const int njobs = ns + nrot;
    const size_t off_jobs = cv.take((size_t)njobs * sizeof(TraceJob));
    // the queue's size once the rotated-S0 jobs are counted (device)
    const size_t off_total = cv.take(sizeof(int64_t));
    // FP64 pass of the FP32 form: re-trace list, its counter, and FP64 node records
    // when a field is stored in FP64 (FP32 records of an FP32 field are exact)
    const bool fixup = P.precision == FQ_PREC_F32X && P.graze > 0;
    int fix_store = FQ_DT_F32;
    for (int i = 0; i < ns; i++)
        if (specs[i].f->dtype == FQ_DT_F64) fix_store = FQ_DT_F64;
    int64_t all_lines = 0;
    for (int i = 0; i < ns; i++) all_lines += W[i].nlines * (W[i].rotate ? 5 : 1);
    size_t off_list = 0, off_lcount = 0, off_jobs64 = 0, off_fkey = 0, off_fcnt = 0, off_flist = 0;
    if (fixup) {
        off_list = cv.take((size_t)(2 * all_lines) * sizeof(FixEntry));
        off_lcount = cv.take(2 * sizeof(uint32_t));  // positions-only and twist lists
        if (P.in_flight) {
            // the positions-only list ordered longest first (keys, counts, the list)
            off_fkey = cv.take((size_t)(2 * all_lines) * sizeof(int32_t));
            off_fcnt = cv.take(256 * sizeof(uint32_t));
            off_flist = cv.take((size_t)(2 * all_lines) * sizeof(FixEntry));
        }
        if (fix_store == FQ_DT_F64) {
            off_jobs64 = cv.take((size_t)njobs * sizeof(TraceJob));
            for (int i = 0; i < ns; i++) {
                const int64_t nn = nodes_of(specs[i].f);
                W[i].nodes64 = cv.take((size_t)nn * (P.want_tw ? 8 : 4) * 8);
            }
        }
    }
    // adjoint: checkpoints, per-half adjoints, node gradients and replay buffers
    size_t off_tape = 0, off_tl = 0, off_tn = 0, off_ta = 0, off_lam = 0, off_ltw = 0, off_gnode = 0;
    size_t off_buf = 0, off_bkey = 0, off_border = 0, off_bcnt = 0, off_lseed = 0;
    int64_t bwd_halves = 0, bwd_nodes = 0;
    if (bwd) {
        // one seed plane or voxel map; an interior plane and a voxel map add their
        // rotated-S0 job (up to four lines per point), whose half lines follow theirs
        if (ns != 1 || nrot > 1 || (specs[0].kind != SPEC_PLANE && specs[0].kind != SPEC_VOXELS))
            return FQ_EUNSUPPORTED;
        if (W[0].rotate && P.scheme != FQ_SCHEME_RKF45) return FQ_EUNSUPPORTED;
        bwd_halves = 2 * W[0].nlines + (W[0].rotate ? 2 * 4 * W[0].nlines : 0);
        bwd_nodes = nodes_of(specs[0].f);
        off_tape = cv.take((size_t)bwd->pool * sizeof(Ckpt));
        off_tl = cv.take((size_t)bwd_halves * sizeof(int32_t));
        off_tn = cv.take((size_t)bwd_halves * sizeof(int32_t));
        off_ta = cv.take((size_t)bwd_halves * sizeof(int32_t));
        off_lam = cv.take((size_t)bwd_halves * 3 * sizeof(double));
        off_ltw = cv.take((size_t)bwd_halves * sizeof(double));
        off_gnode = cv.take((size_t)bwd_nodes * (P.want_tw ? 6 : 3) * sizeof(double));
        off_buf = cv.take((size_t)kBwdSlots * (size_t)bwd->seg * sizeof(StepRec));
        off_bkey = cv.take((size_t)bwd_halves * sizeof(int32_t));
        off_border = cv.take((size_t)bwd_halves * sizeof(int32_t));
        if (W[0].rotate) off_lseed = cv.take((size_t)2 * 4 * W[0].nlines * 3 * sizeof(double));
        off_bcnt = cv.take(256 * sizeof(uint32_t));
    }
    if (need) *need = cv.off;
    if (dry) return FQ_OK;
    if (!ws) return FQ_EINVAL;
    if (ws_bytes < cv.off) return FQ_ENOMEM;
    if (((uintptr_t)ws & 255) != 0) return FQ_EINVAL;

    hipError_t e = hipSuccess;
#define FQ_TRY(x)                      \
    do {                               \
        e = (x);                       \
        if (e != hipSuccess) return FQ_EHIP; \
    } while (0)

    // the kernels of the forward pass (all but the reverse of a recorded forward pass)
    // and of the reverse pass
    const bool fwd = !bwd || bwd->phase != 2;
    const bool rev = bwd && bwd->phase != 1;
    unsigned long long *counter = (unsigned long long *)(ws + off_ctr);
    if (fwd) FQ_TRY(launch_fill_u32((uint32_t *)(ws + off_ctr), 4, 0u, stream));
    for (int i = 0; i < ns && fwd; i++) {
        const Spec &s = specs[i];
        SpecWs &w = W[i];
        FQ_TRY(launch_fill_u32((uint32_t *)(ws + w.bmax), 1, 0u, stream));
        if (w.rotate) FQ_TRY(launch_fill_u32((uint32_t *)(ws + w.rot_count), 1, 0u, stream));
        if (stretched(s.f)) {
            double *const iw[3] = {(double *)(ws + w.iw[0]), (double *)(ws + w.iw[1]),
                                   (double *)(ws + w.iw[2])};
            FQ_TRY(launch_geometry(*s.f, iw, (Geo *)(ws + w.geo), stream));
        }
        FQ_TRY(launch_prep(*s.f, P.precision, P.want_tw, ws + w.nodes, (float *)(ws + w.bmax), stream));
        if (fixup && fix_store == FQ_DT_F64)
            FQ_TRY(launch_prep(*s.f, FQ_PREC_F64, P.want_tw, ws + w.nodes64, (float *)(ws + w.bmax),
                               stream));
    }
    // rotated-S0 classification (each map with an interior S0)
    std::vector<MapJob> maps(ns);
    for (int i = 0; i < ns; i++) {
        const Spec &s = specs[i];
        SpecWs &w = W[i];
        MapJob &m = maps[i];
        memset(&m, 0, sizeof m);
        set_map_geometry(s, m);
        m.edge_eps = P.edge_eps;
        m.rec = recs_at(ws, w.end, w.tw, w.len, w.face, w.st);
        if (m2) m.rec.uv = (double *)(ws + w.uv);
        m.nlines = w.nlines;
        if (s.kind != SPEC_LIST && s.map) m.out = *s.map;
        if (s.kind == SPEC_LIST && s.lines) m.out.lines = *s.lines;
        if (w.rotate) {
            m.rot_index = (const int32_t *)(ws + w.rot_index);
            m.rot = (const RotEntry *)(ws + w.rot);
            m.rot_rec = recs_at(ws, w.r_end, w.r_tw, w.r_len, w.r_face, w.r_st);
            m.rot_nlines = 4 * w.nlines;
            m.rot_delta = fmin(m.d0, m.d1);
            // (the reverse of a recorded forward pass reads the classification it left)
            if (fwd)
                FQ_TRY(launch_classify(m, (int32_t *)(ws + w.rot_index), (RotEntry *)(ws + w.rot),
                                       (uint32_t *)(ws + w.rot_count), w.nlines, stream));
        }
    }
    // job table
    std::vector<TraceJob> jobs(njobs);
    int64_t items = 0;
    int jj = 0;
    for (int i = 0; i < ns; i++) {
        const Spec &s = specs[i];
        SpecWs &w = W[i];
        TraceJob &J = jobs[jj++];
        memset(&J, 0, sizeof J);
        J.nodes = ws + w.nodes;
        J.bmax2 = (const float *)(ws + w.bmax);
        for (int a = 0; a < 3; a++) {
            J.n[a] = (int32_t)s.f->n[a];
            J.origin[a] = s.f->origin[a];
            J.spacing[a] = s.f->spacing[a];
            J.normal[a] = s.normal[a];
        }
        J.nlines = w.nlines;
        J.rec = recs_at(ws, w.end, w.tw, w.len, w.face, w.st);
        if (m2) J.rec.uv = (double *)(ws + w.uv);
        for (int a = 0; a < 3; a++) {
            J.planes.b[a] = s.f->b[a];
            J.planes.n[a] = (int32_t)s.f->n[a];
            J.planes.origin[a] = s.f->origin[a];
            J.planes.spacing[a] = s.f->spacing[a];
            J.planes.coord[a] = s.f->coord[a];
        }
        J.planes.dtype = s.f->dtype;
        if (stretched(s.f)) {
            for (int a = 0; a < 3; a++) J.iw[a] = (const double *)(ws + w.iw[a]);
            J.geo = (const Geo *)(ws + w.geo);
        }
        if (s.kind == SPEC_LIST) {
            J.kind = SEED_LIST;
            J.seeds = s.seeds;
            J.tile[0] = 64, J.tile[1] = 1, J.tile[2] = 1;
            J.dims[0] = s.nlist, J.dims[1] = 1, J.dims[2] = 1;
        } else if (s.kind == SPEC_PLANE) {
            J.kind = SEED_PLANE;
            J.tile[0] = 8, J.tile[1] = 8, J.tile[2] = 1;
            J.dims[0] = s.pl.nu, J.dims[1] = s.pl.nv, J.dims[2] = 1;
            for (int a = 0; a < 3; a++) {
                J.s_origin[a] = s.pl.origin[a];
                J.s_a[a] = s.pl.du * s.pl.u[a];
                J.s_b[a] = s.pl.dv * s.pl.v[a];
            }
        } else if (s.kind == SPEC_CYL) {
            J.kind = SEED_CYL;
            J.tile[0] = 8, J.tile[1] = 8, J.tile[2] = 1;
            J.dims[0] = s.cy.ntheta, J.dims[1] = s.cy.nz, J.dims[2] = 1;
            J.cyl[0] = s.cy.centre[0];
            J.cyl[1] = s.cy.centre[1];
            J.cyl[2] = s.cy.radius;
            J.s_origin[0] = s.cy.theta0;
            J.s_a[0] = s.cy.dtheta;
            J.s_origin[1] = s.cy.z0;
            J.s_b[1] = s.cy.dz;
        } else {
            J.kind = SEED_VOXELS;
            J.tile[0] = 4, J.tile[1] = 4, J.tile[2] = 4;
            for (int a = 0; a < 3; a++) {
                J.dims[a] = s.vx.n[a];
                J.s_origin[a] = s.vx.origin[a];
            }
            J.s_a[0] = s.vx.spacing[0];
            J.s_b[1] = s.vx.spacing[1];
            J.s_c[2] = s.vx.spacing[2];
        }
        int64_t tv = 1;
        for (int a = 0; a < 3; a++) {
            J.tiles[a] = (J.dims[a] + J.tile[a] - 1) / J.tile[a];
            tv *= J.tiles[a] * J.tile[a];
        }
        J.nitems = tv;
        set_job_constants(J);
        if (s.kind == SPEC_PLANE) {
            J.tile_order = (const int32_t *)(ws + w.tile_order);
            if (fwd)
                FQ_TRY(launch_tile_order(J, P.precision, P.want_tw, (int32_t *)(ws + w.tile_bucket), (uint32_t *)(ws + w.tile_counts),
                                         (int32_t *)(ws + w.tile_order), stream));
        } else if (s.kind == SPEC_VOXELS) {
            J.tile_order = (const int32_t *)(ws + w.tile_order);
            if (fwd)
                FQ_TRY(launch_voxel_order(J, P.precision, P.want_tw, (int32_t *)(ws + w.tile_bucket),
                                          (uint32_t *)(ws + w.tile_counts), (int32_t *)(ws + w.tile_order),
                                          stream));
        }
    }
    // queue ranges of the main jobs, largest cube first: its lines reach farthest, so
    // they start early (inside a job, plane tiles follow their own length order)
    {
        std::vector<int> perm(ns);
        for (int i = 0; i < ns; i++) perm[i] = i;
        auto edge = [&](int i) {
            const int64_t *n = specs[i].f->n;
            return n[0] > n[1] ? (n[0] > n[2] ? n[0] : n[2]) : (n[1] > n[2] ? n[1] : n[2]);
        };
        std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) { return edge(x) > edge(y); });
        for (int k = 0; k < ns; k++) {
            TraceJob &J = jobs[perm[k]];
            J.item_base = items;
            items += 2 * J.nitems;
        }
    }
    TraceParams tp;
    memset(&tp, 0, sizeof tp);
    std::vector<int> rot_spec;  // the spec of each rotated-S0 job (jobs ns, ns + 1, ...)
    for (int i = 0; i < ns; i++) {
        if (!W[i].rotate) continue;
        const SpecWs &w = W[i];
        rot_spec.push_back(i);
        TraceJob &J = jobs[jj++];
        J = jobs[i];
        J.kind = SEED_ROTATED;
        J.tile_order = nullptr;
        J.seeds = nullptr;
        J.rot = (const RotEntry *)(ws + w.rot);
        J.rot_count = (const uint32_t *)(ws + w.rot_count);
        J.rot_delta = maps[i].rot_delta;
        J.nlines = 4 * w.nlines;
        J.tile[0] = 64, J.tile[1] = 1, J.tile[2] = 1;
        J.dims[0] = 4 * w.nlines, J.dims[1] = 1, J.dims[2] = 1;
        J.tiles[0] = (J.dims[0] + 63) / 64, J.tiles[1] = 1, J.tiles[2] = 1;
        J.nitems = J.tiles[0] * 64;
        set_job_constants(J);
        J.rec = recs_at(ws, w.r_end, w.r_tw, w.r_len, w.r_face, w.r_st);
        J.item_base = items;
        tp.dynamic_last = 1;
    }
    TraceJob *jobs_dev = (TraceJob *)(ws + off_jobs);
    for (int j = 0; j < njobs && fwd; j++) FQ_TRY(launch_store_job(jobs[j], jobs_dev + j, stream));
    if (nrot > 0 && fwd)
        FQ_TRY(launch_rot_ranges(jobs_dev, ns, nrot, items, (int64_t *)(ws + off_total), stream));
    tp.total_dev = (const int64_t *)(ws + off_total);
    tp.tol_perp = P.tol_perp;
    tp.step_perp = P.step_perp;
    tp.step_min = P.step_min;
    tp.tol_floor = P.tol_floor;
    tp.scheme = P.scheme;
    tp.method = m2 ? FQ_METHOD_II : FQ_METHOD_I;
    for (int i = 0; i < ns; i++) {
        if (stretched(specs[i].f)) tp.stretched = 1;
        if (specs[i].kind == SPEC_CYL) tp.cyl = 1;
    }
    tp.max_steps = P.max_steps;
    tp.want_tw = P.want_tw;
    tp.njobs = njobs;
    if (xcd) {
        tp.xcd_ctr = (unsigned long long *)(ws + off_xctr);
        if (fwd) FQ_TRY(launch_fill_u32((uint32_t *)(ws + off_xctr), 128, 0u, stream));
    }
    tp.stats = bwd ? nullptr : (unsigned long long *)P.stats;
    tp.static_items = items;
    if (bwd) {
        tp.tape = (Ckpt *)(ws + off_tape);
        tp.pool_ctr = (unsigned long long *)(ws + off_ctr + 128);
        tp.tape_last = (int32_t *)(ws + off_tl);
        tp.tape_n = (int32_t *)(ws + off_tn);
        tp.tape_acc = (int32_t *)(ws + off_ta);
        tp.seg = bwd->seg;
        tp.pool_cap = bwd->pool;
        tp.tape_base1 = 2 * W[0].nlines;
        if (fwd) FQ_TRY(launch_fill_u32((uint32_t *)(ws + off_ctr + 128), 2, 0u, stream));
    }
    hipEvent_t *ev = fwd ? (hipEvent_t *)P.events : nullptr;
    if (ev && ev[0]) FQ_TRY(hipEventRecord(ev[0], stream));
    if (fwd)
        FQ_TRY(launch_trace(P.precision, P.precision == FQ_PREC_F64 ? FQ_DT_F64 : FQ_DT_F32, P.want_tw,
                            jobs_dev, tp, counter, P.block, P.waves_per_cu, stream));
    if (ev && ev[1]) FQ_TRY(hipEventRecord(ev[1], stream));
    if (fixup && fwd) {
        // FP64 pass over the grazing lines of the FP32 pass, and over the lines whose
        // map point has a large Q by the FP32 pass (formed here first)
        const bool qsel = P.qfix > 0;
        if (qsel)
            for (int i = 0; i < ns; i++) {
                if (specs[i].kind == SPEC_LIST || !maps[i].out.q) continue;
                MapJob mq = maps[i];  // Q only: the final pass writes every output
                memset(&mq.out, 0, sizeof mq.out);
                mq.out.q = maps[i].out.q;
                FQ_TRY(specs[i].kind == SPEC_CYL ? launch_cyl_map(mq, stream)
                       : m2                     ? launch_m2_map(mq, stream)
                                                : launch_stencil(mq, stream));
            }
        // Method I keeps the FP32 pass's twist and re-traces positions only, then the
        // half lines that pass could not finish with the twist (split lists); Method
        // II has no positions-only tracer and re-traces everything in one list
        const bool split = P.want_tw && !m2;
        FixEntry *list = (FixEntry *)(ws + off_list);
        uint32_t *lcount = (uint32_t *)(ws + off_lcount);
        FQ_TRY(launch_fill_u32(lcount, 2, 0u, stream));
        FQ_TRY(launch_fill_u32((uint32_t *)(ws + off_ctr), 2, 0u, stream));
        for (int j = 0; j < njobs; j++) {
            // the spec whose map decides the Q rule: a main job's own, or for the
            // rotated-S0 job the map of the spec it belongs to
            const int sp = j < ns ? j : rot_spec[j - ns];
            const double *qmap = (qsel && specs[sp].kind != SPEC_LIST) ? maps[sp].out.q : nullptr;
            FQ_TRY(launch_graze(jobs_dev, j, jobs[j].nlines, P.graze, qmap, P.qfix, list, lcount,
                                lcount + 1, 2 * all_lines, split, !m2, stream));
        }
        const TraceJob *fix_jobs = jobs_dev;
        if (fix_store == FQ_DT_F64) {
            TraceJob *j64 = (TraceJob *)(ws + off_jobs64);
            int k = 0;
            for (int i = 0; i < ns; i++) {
                TraceJob J = jobs[i];
                J.nodes = ws + W[i].nodes64;
                FQ_TRY(launch_store_job(J, j64 + k++, stream));
            }
            for (int i = 0; i < ns; i++) {
                if (!W[i].rotate) continue;
                TraceJob J = jobs[k];
                J.nodes = ws + W[i].nodes64;
                FQ_TRY(launch_store_job(J, j64 + k++, stream));
            }
            fix_jobs = j64;
        }
        TraceParams fp = tp;
        fp.tape = nullptr;  // the adjoint's checkpoints come from the FP32 pass only
        fp.xcd_ctr = nullptr;  // list mode: one queue
        fp.list = list;
        if (P.in_flight) {
            // with other maps in flight, a wave that holds lines of like length frees its
            // SIMD slot for them sooner: the list longest first
            FixEntry *sorted = (FixEntry *)(ws + off_flist);
            FQ_TRY(launch_fix_order(jobs_dev, list, lcount, 2 * all_lines, (int32_t *)(ws + off_fkey),
                                    (uint32_t *)(ws + off_fcnt), sorted, stream));
            fp.list = sorted;
        }
        fp.list_count = lcount;
        fp.list_cap = 2 * all_lines;
        // the FP64 pass is held to the FP64 floor unless the caller set a larger one
        fp.tol_floor = P.tol_floor == kFloor32 ? kFloor64 : P.tol_floor;
        if (ev && ev[2]) FQ_TRY(hipEventRecord(ev[2], stream));
        // positions only: the twist integral is not sensitive to the end angle, so the
        // FP32 pass's Tw is kept and the latency-bound FP64 pass skips the curl
        // (with other maps in flight, the positions-only form at three waves per SIMD)
        const int fix_twm = !P.want_tw ? 0 : (split ? (P.in_flight ? 3 : 2) : 1);
        FQ_TRY(launch_trace(FQ_PREC_F64, fix_store, fix_twm, fix_jobs, fp, counter, P.block,
                            P.waves_per_cu, stream));
        if (split) {
            // half lines the FP32 pass could not finish have no twist yet: trace those
            // (usually none) with the twist integrand, on a queue counter of their own
            TraceParams ft = fp;
            ft.list = list;  // the twist list sits at the top of the unordered array
            ft.list_count = lcount + 1;
            ft.list_rev = 1;
            unsigned long long *c2 = (unsigned long long *)(ws + off_ctr + 192);
            FQ_TRY(launch_fill_u32((uint32_t *)c2, 2, 0u, stream));
            FQ_TRY(launch_trace(FQ_PREC_F64, fix_store, 1, fix_jobs, ft, c2, P.block, P.waves_per_cu,
                                stream));
        }
        if (ev && ev[3]) FQ_TRY(hipEventRecord(ev[3], stream));
    }
    if (rev) {
        double *lam_end = (double *)(ws + off_lam), *lam_tw = (double *)(ws + off_ltw);
        double *gnode = (double *)(ws + off_gnode);
        FQ_TRY(launch_fill_u32((uint32_t *)lam_end, bwd_halves * 6, 0u, stream));
        FQ_TRY(launch_fill_u32((uint32_t *)lam_tw, bwd_halves * 2, 0u, stream));
        FQ_TRY(launch_fill_u32((uint32_t *)gnode, bwd_nodes * (P.want_tw ? 12 : 6), 0u, stream));
        FQ_TRY(launch_map_backward(maps[0], bwd->dq, P.want_tw ? bwd->dtw : nullptr, bwd->dend_b,
                                   bwd->dend_f, lam_end, lam_tw, gnode, 2 * W[0].nlines, stream));
        unsigned long long *bctr = (unsigned long long *)(ws + off_ctr + 64);
        FQ_TRY(launch_fill_u32((uint32_t *)bctr, 2, 0u, stream));
        BwdParams bp;
        memset(&bp, 0, sizeof bp);
        bp.tape = tp.tape;
        bp.tape_last = tp.tape_last;
        bp.tape_n = tp.tape_n;
        bp.tape_acc = tp.tape_acc;
        bp.seg = tp.seg;
        bp.nhalves = bwd_halves;
        bp.nhalf0 = 2 * W[0].nlines;
        double *lseed = W[0].rotate ? (double *)(ws + off_lseed) : nullptr;
        if (lseed) FQ_TRY(launch_fill_u32((uint32_t *)lseed, 2 * 4 * W[0].nlines * 6, 0u, stream));
        bp.lam_seed = lseed;
        bp.lam_end = lam_end;
        bp.lam_tw = lam_tw;
        bp.gnode = gnode;
        bp.buf = (StepRec *)(ws + off_buf);
        bp.nslots = kBwdSlots;
        bp.counter = bctr;
        int32_t *border = (int32_t *)(ws + off_border);
        FQ_TRY(launch_bwd_order(tp.tape_acc, bwd_halves, (int32_t *)(ws + off_bkey),
                                (uint32_t *)(ws + off_bcnt), border, stream));
        bp.order = border;
        bp.stats = (unsigned long long *)P.stats;
        bp.max_steps = P.max_steps;
        bp.want_tw = P.want_tw;
        bp.scheme = P.scheme;
        // the reverse pass replays the forward pass's steps in its own arithmetic: FP64
        // records and FP64 steps, or the F32X form's FP32 records and FP32 pass
        FQ_TRY(launch_trace_backward(P.precision == FQ_PREC_F64 ? FQ_DT_F64 : FQ_DT_F32, P.want_tw,
                                     jobs_dev, bp, stream));
        if (lseed)
            FQ_TRY(launch_rot_seed(maps[0], (const RotEntry *)(ws + W[0].rot),
                                   (const uint32_t *)(ws + W[0].rot_count), W[0].nlines, lseed, gnode,
                                   stream));
        FQ_TRY(launch_grad_planes(*specs[0].f, gnode, P.want_tw, bwd->gb, stream));
        return FQ_OK;
    }
    for (int i = 0; i < ns; i++) {
        if (specs[i].kind == SPEC_LIST) FQ_TRY(launch_lines_out(maps[i], specs[i].seeds, stream));
        else if (specs[i].kind == SPEC_CYL) FQ_TRY(launch_cyl_map(maps[i], stream));
        else if (m2) FQ_TRY(launch_m2_map(maps[i], stream));
        else FQ_TRY(launch_stencil(maps[i], stream));
        // Q_perp by Method I (plane maps) and the length edge map (plane maps, both
        // methods)
        if (specs[i].kind == SPEC_PLANE && (maps[i].out.fledge || (!m2 && maps[i].out.qperp)))
            FQ_TRY(launch_perp_map(maps[i], !m2, stream));
    }
#undef FQ_TRY
    return FQ_OK;
}

// Constants the tracer would otherwise recompute per half line.
void set_job_constants(TraceJob &J)
{
    const double dm = fmin(J.spacing[0], fmin(J.spacing[1], J.spacing[2]));
    for (int a = 0; a < 3; a++) J.rscale[a] = (float)(dm / J.spacing[a]);
    J.twk = (float)(dm / (4.0 * M_PI));
    J.dref = dm;
    for (int a = 0; a < 3; a++) J.inv_spacing[a] = 1.0 / J.spacing[a];
    J.inv_t0 = 1.0 / (double)J.tiles[0];
    J.inv_t1 = 1.0 / (double)J.tiles[1];
}

void plane_normal(const fq_plane &p, double n[3])
{
    n[0] = p.u[1] * p.v[2] - p.u[2] * p.v[1];
    n[1] = p.u[2] * p.v[0] - p.u[0] * p.v[2];
    n[2] = p.u[0] * p.v[1] - p.u[1] * p.v[0];
}

int q2d_specs(const fq_field *fields, const fq_plane *planes, int njobs, const fq_map *maps,
              std::vector<Spec> &specs)
{
    if (njobs < 1 || !fields || !planes) return FQ_EINVAL;
    specs.resize(njobs);
    for (int j = 0; j < njobs; j++) {
        int rc = check_field(&fields[j]);
        if (rc) return rc;
        if ((rc = check_plane(&planes[j]))) return rc;
        Spec &s = specs[j];
        memset(&s, 0, sizeof s);
        s.kind = SPEC_PLANE;
        s.f = &fields[j];
        s.pl = planes[j];
        plane_normal(planes[j], s.normal);
        s.map = maps ? &maps[j] : nullptr;
    }
    return FQ_OK;
}

// What every adjoint call checks, and its checkpoint pool: room for tape_steps
// accepted steps per half line of the seed points on average (plus the first
// checkpoint and a partial segment), and where points may take a rotated S0 those two
// for each potential half line of its job (its lines, where a point has them, share
// the points' average)
int bwd_common(const fq_params *p, int segment, int64_t points, bool rotated, fq_params &P,
               BwdSpec &b)
{
    int rc = resolve_params(p, P);
    if (rc) return rc;
    if (P.method != FQ_METHOD_I) return FQ_EUNSUPPORTED;
    if (segment < 1 || segment > 4096) return FQ_EINVAL;
    if (P.max_steps > INT32_MAX) return FQ_EINVAL;
    memset(&b, 0, sizeof b);
    b.seg = segment;
    const int64_t halves = 2 * points;
    if (P.tape_steps > ((int64_t)1 << 40)) return FQ_EINVAL;
    b.pool = halves * (2 + (P.tape_steps + segment - 1) / segment);
    if (rotated) b.pool += 4 * halves * 2;
    if (b.pool > INT32_MAX) return FQ_EINVAL;
    return FQ_OK;
}

int bwd_setup(const fq_field *f, const fq_plane *pl, const fq_params *p, int segment,
              fq_params &P, std::vector<Spec> &v, BwdSpec &b)
{
    int rc = resolve_params(p, P);
    if (rc) return rc;
    if ((rc = check_field(f)) || (rc = check_plane(pl))) return rc;
    if ((rc = bwd_common(p, segment, pl->nu * pl->nv, !plane_on_face(*pl, *f), P, b))) return rc;
    return q2d_specs(f, pl, 1, nullptr, v);
}

// A 3-D map's adjoint: its voxel layers are seed planes whose points may all take a
// rotated S0.
int bwd_setup_vx(const fq_field *f, const fq_voxels *vx, const fq_params *p, int segment,
                 fq_params &P, std::vector<Spec> &v, BwdSpec &b)
{
    int rc = resolve_params(p, P);
    if (rc) return rc;
    if ((rc = check_field(f)) || (rc = check_voxels(vx))) return rc;
    if ((rc = bwd_common(p, segment, vx->n[0] * vx->n[1] * vx->n[2], true, P, b))) return rc;
    Spec s;
    memset(&s, 0, sizeof s);
    s.kind = SPEC_VOXELS;
    s.f = f;
    s.vx = *vx;
    s.normal[2] = 1.0;
    v.assign(1, s);
    return FQ_OK;
}

}  // namespace
}  // namespace fq

using namespace fq;

extern "C" {

const char *fastqsl_version(void) { return "fastqsl-mi355x 0.1 (gfx950)"; }

const char *fastqsl_strerror(int code)
{
    switch (code) {
    case FQ_OK: return "ok";
    case FQ_EINVAL: return "invalid argument";
    case FQ_ENOMEM: return "workspace too small";
    case FQ_EHIP: return "HIP launch failed";
    case FQ_EUNSUPPORTED: return "unsupported combination";
    default: return "unknown error";
    }
}

size_t fastqsl_trace_workspace_size(const fq_field *f, int64_t n, const fq_params *p)
{
    fq_params P;
    if (resolve_params(p, P) || check_field(f) || n < 0) return 0;
    Spec s;
    memset(&s, 0, sizeof s);
    s.kind = SPEC_LIST;
    s.f = f;
    s.nlist = n;
    std::vector<Spec> v(1, s);
    size_t need = 0;
    run(v, P, nullptr, 0, true, &need, nullptr);
    return need;
}

int fastqsl_trace(const fq_field *f, const double *seeds, int64_t n, const double *normal,
                  const fq_params *p, const fq_lines *out, void *ws, size_t ws_bytes,
                  void *stream)
{
    fq_params P;
    int rc = resolve_params(p, P);
    if (rc) return rc;
    if ((rc = check_field(f))) return rc;
    if (n < 0 || (n > 0 && !seeds) || !out) return FQ_EINVAL;
    if (n == 0) return FQ_OK;
    Spec s;
    memset(&s, 0, sizeof s);
    s.kind = SPEC_LIST;
    s.f = f;
    s.seeds = seeds;
    s.nlist = n;
    s.lines = out;
    if (normal) {
        double nn = sqrt(normal[0] * normal[0] + normal[1] * normal[1] + normal[2] * normal[2]);
        if (!(nn > 0.0) || !isfinite(nn)) return FQ_EINVAL;
        for (int a = 0; a < 3; a++) s.normal[a] = normal[a] / nn;
    } else {
        s.normal[2] = 1.0;
    }
    std::vector<Spec> v(1, s);
    return run(v, P, (char *)ws, ws_bytes, false, nullptr, (hipStream_t)stream);
}

size_t fastqsl_q2d_workspace_size(const fq_field *fields, const fq_plane *planes, int njobs,
                                  const fq_params *p)
{
    fq_params P;
    std::vector<Spec> v;
    if (resolve_params(p, P) || q2d_specs(fields, planes, njobs, nullptr, v)) return 0;
    size_t need = 0;
    if (run(v, P, nullptr, 0, true, &need, nullptr)) return 0;
    return need;
}

int fastqsl_q2d(const fq_field *fields, const fq_plane *planes, int njobs, const fq_params *p,
                const fq_map *maps, void *ws, size_t ws_bytes, void *stream)
{
    fq_params P;
    int rc = resolve_params(p, P);
    if (rc) return rc;
    if (!maps) return FQ_EINVAL;
    std::vector<Spec> v;
    if ((rc = q2d_specs(fields, planes, njobs, maps, v))) return rc;
    return run(v, P, (char *)ws, ws_bytes, false, nullptr, (hipStream_t)stream);
}

size_t fastqsl_q3d_workspace_size(const fq_field *f, const fq_voxels *vx, const fq_params *p)
{
    fq_params P;
    if (resolve_params(p, P) || check_field(f) || check_voxels(vx)) return 0;
    Spec s;
    memset(&s, 0, sizeof s);
    s.kind = SPEC_VOXELS;
    s.f = f;
    s.vx = *vx;
    s.normal[2] = 1.0;
    std::vector<Spec> v(1, s);
    size_t need = 0;
    run(v, P, nullptr, 0, true, &need, nullptr);
    return need;
}

int fastqsl_q3d(const fq_field *f, const fq_voxels *vx, const fq_params *p, const fq_map *map,
                void *ws, size_t ws_bytes, void *stream)
{
    fq_params P;
    int rc = resolve_params(p, P);
    if (rc) return rc;
    if ((rc = check_field(f)) || (rc = check_voxels(vx))) return rc;
    if (!map) return FQ_EINVAL;
    Spec s;
    memset(&s, 0, sizeof s);
    s.kind = SPEC_VOXELS;
    s.f = f;
    s.vx = *vx;
    s.normal[2] = 1.0;
    s.map = map;
    std::vector<Spec> v(1, s);
    return run(v, P, (char *)ws, ws_bytes, false, nullptr, (hipStream_t)stream);
}

size_t fastqsl_qcyl_workspace_size(const fq_field *f, const fq_cylinder *c, const fq_params *p)
{
    fq_params P;
    if (resolve_params(p, P) || check_field(f) || check_cylinder(c, f)) return 0;
    Spec s;
    memset(&s, 0, sizeof s);
    s.kind = SPEC_CYL;
    s.f = f;
    s.cy = *c;
    std::vector<Spec> v(1, s);
    size_t need = 0;
    if (run(v, P, nullptr, 0, true, &need, nullptr)) return 0;
    return need;
}

int fastqsl_qcyl(const fq_field *f, const fq_cylinder *c, const fq_params *p, const fq_map *map,
                 void *ws, size_t ws_bytes, void *stream)
{
    fq_params P;
    int rc = resolve_params(p, P);
    if (rc) return rc;
    if ((rc = check_field(f)) || (rc = check_cylinder(c, f))) return rc;
    if (!map) return FQ_EINVAL;
    Spec s;
    memset(&s, 0, sizeof s);
    s.kind = SPEC_CYL;
    s.f = f;
    s.cy = *c;
    s.map = map;
    std::vector<Spec> v(1, s);
    return run(v, P, (char *)ws, ws_bytes, false, nullptr, (hipStream_t)stream);
}

size_t fastqsl_backward_workspace_size(const fq_field *f, const fq_plane *pl, const fq_params *p,
                                       int segment)
{
    fq_params P;
    std::vector<Spec> v;
    BwdSpec b;
    if (bwd_setup(f, pl, p, segment, P, v, b)) return 0;
    size_t need = 0;
    if (run(v, P, nullptr, 0, true, &need, nullptr, &b)) return 0;
    return need;
}

int fastqsl_backward(const fq_field *f, const fq_plane *pl, const fq_params *p, int segment,
                     const double *dq, const double *dtw, const double *dend_b,
                     const double *dend_f, double *const gb[3], void *ws, size_t ws_bytes,
                     void *stream)
{
    fq_params P;
    std::vector<Spec> v;
    BwdSpec b;
    int rc = bwd_setup(f, pl, p, segment, P, v, b);
    if (rc) return rc;
    if (!gb || !gb[0] || !gb[1] || !gb[2]) return FQ_EINVAL;
    b.dq = dq;
    b.dtw = dtw;
    b.dend_b = dend_b;
    b.dend_f = dend_f;
    b.gb = gb;
    return run(v, P, (char *)ws, ws_bytes, false, nullptr, (hipStream_t)stream, &b);
}

int fastqsl_q2d_record(const fq_field *f, const fq_plane *pl, const fq_params *p, int segment,
                       const fq_map *map, void *ws, size_t ws_bytes, void *stream)
{
    fq_params P;
    std::vector<Spec> v;
    BwdSpec b;
    int rc = bwd_setup(f, pl, p, segment, P, v, b);
    if (rc) return rc;
    if (!map) return FQ_EINVAL;
    v[0].map = map;
    b.phase = 1;
    return run(v, P, (char *)ws, ws_bytes, false, nullptr, (hipStream_t)stream, &b);
}

int fastqsl_backward_recorded(const fq_field *f, const fq_plane *pl, const fq_params *p,
                              int segment, const double *dq, const double *dtw,
                              const double *dend_b, const double *dend_f, double *const gb[3],
                              void *ws, size_t ws_bytes, void *stream)
{
    fq_params P;
    std::vector<Spec> v;
    BwdSpec b;
    int rc = bwd_setup(f, pl, p, segment, P, v, b);
    if (rc) return rc;
    if (!gb || !gb[0] || !gb[1] || !gb[2]) return FQ_EINVAL;
    b.dq = dq;
    b.dtw = dtw;
    b.dend_b = dend_b;
    b.dend_f = dend_f;
    b.gb = gb;
    b.phase = 2;
    return run(v, P, (char *)ws, ws_bytes, false, nullptr, (hipStream_t)stream, &b);
}

size_t fastqsl_q3d_backward_workspace_size(const fq_field *f, const fq_voxels *vx,
                                           const fq_params *p, int segment)
{
    fq_params P;
    std::vector<Spec> v;
    BwdSpec b;
    if (bwd_setup_vx(f, vx, p, segment, P, v, b)) return 0;
    size_t need = 0;
    if (run(v, P, nullptr, 0, true, &need, nullptr, &b)) return 0;
    return need;
}

int fastqsl_q3d_backward(const fq_field *f, const fq_voxels *vx, const fq_params *p, int segment,
                         const double *dq, const double *dtw, const double *dend_b,
                         const double *dend_f, double *const gb[3], void *ws, size_t ws_bytes,
                         void *stream)
{
    fq_params P;
    std::vector<Spec> v;
    BwdSpec b;
    int rc = bwd_setup_vx(f, vx, p, segment, P, v, b);
    if (rc) return rc;
    if (!gb || !gb[0] || !gb[1] || !gb[2]) return FQ_EINVAL;
    b.dq = dq;
    b.dtw = dtw;
    b.dend_b = dend_b;
    b.dend_f = dend_f;
    b.gb = gb;
    return run(v, P, (char *)ws, ws_bytes, false, nullptr, (hipStream_t)stream, &b);
}

int fastqsl_q3d_record(const fq_field *f, const fq_voxels *vx, const fq_params *p, int segment,
                       const fq_map *map, void *ws, size_t ws_bytes, void *stream)
{
    fq_params P;
    std::vector<Spec> v;
    BwdSpec b;
    int rc = bwd_setup_vx(f, vx, p, segment, P, v, b);
    if (rc) return rc;
    if (!map) return FQ_EINVAL;
    v[0].map = map;
    b.phase = 1;
    return run(v, P, (char *)ws, ws_bytes, false, nullptr, (hipStream_t)stream, &b);
}

int fastqsl_q3d_backward_recorded(const fq_field *f, const fq_voxels *vx, const fq_params *p,
                                  int segment, const double *dq, const double *dtw,
                                  const double *dend_b, const double *dend_f,
                                  double *const gb[3], void *ws, size_t ws_bytes, void *stream)
{
    fq_params P;
    std::vector<Spec> v;
    BwdSpec b;
    int rc = bwd_setup_vx(f, vx, p, segment, P, v, b);
    if (rc) return rc;
    if (!gb || !gb[0] || !gb[1] || !gb[2]) return FQ_EINVAL;
    b.dq = dq;
    b.dtw = dtw;
    b.dend_b = dend_b;
    b.dend_f = dend_f;
    b.gb = gb;
    b.phase = 2;
    return run(v, P, (char *)ws, ws_bytes, false, nullptr, (hipStream_t)stream, &b);
}

}  // extern "C"
