// Persistent field-line tracer for gfx950.
//
// One lane traces one half line (a seed followed along B or against it) through the
// trilinear field (Section 2.2, Eq. interp) by adaptive RKF45 steps (Section 2.3,
// Fehlberg's 4(5) pair) of dr/ds = B/|B| (Section 2.1, Eq. rb), with the twist
// integrand of Eq. tw (Section 1) and the length as two more ODE components, until
// the line leaves the box (Section 2.1).
//
// Design for CDNA:
//  * Cell-resident interpolation. Inside one grid cell the trilinear interpolant is
//    a polynomial; a lane keeps the current cell's 8 monomial coefficients of
//    B (and of curl B) in VGPRs, so the six RK stages of a step gather nothing.
//    A cell is fetched once per visit: 8 + 8 vector loads of the node records
//    written by the prep pass.
//  * Cell-local coordinates. Position = integer cell + local coordinates in [0,1];
//    FP32 local coordinates keep an absolute resolution of ~1e-7 grid spacings
//    anywhere in a cube of any size, so FP32 integration does not lose the
//    footpoint accuracy to the size of the box.
//  * Exact face landing. Every step stays inside the closed cell (the interpolant
//    has a kink on every cell face, which would otherwise cost the integrator its
//    order). A step that reaches a face is taken with the coordinate normal to that
//    face as the independent variable, so it ends exactly on the face; the line then
//    continues in the neighbouring cell, or ends if the face is a box face.
//  * Persistent lanes and a global queue. Line lengths differ by orders of
//    magnitude; a lane that finishes pops the next half line from a global counter
//    (one atomic per wave via a ballot), so waves never idle on their longest line.
//    Queue items follow 64-seed tiles, so the lanes of a wave start on neighbouring
//    seeds and read neighbouring cells.
#include "fq_internal.h"
#include "trace_core.h"
#include "trace_dev.h"

namespace fq {
namespace {

using namespace dev;

// UNI: a single job without a rotated-S0 companion, so every job constant is
// uniform across the grid (kept in scalar registers).
// TAPE: the adjoint's forward pass (single job; FP64, or the FP32 pass of the F32X
// form), which also stores the lane state at the start of every half line and after
// every tp.seg accepted steps.
template <typename T, int TWM, bool UNI, bool TAPE>
__device__ __forceinline__ bool store_ckpt(const TraceParams &tp, int &last, const Lane<T> &L)
{
    if (!TAPE) return true;
    const unsigned long long slot = atomicAdd(tp.pool_ctr, 1ull);
    if (slot >= (unsigned long long)tp.pool_cap) return false;  // the pool is exhausted
    Ckpt c;
    c.p0 = (double)L.p0;
    c.p1 = (double)L.p1;
    c.p2 = (double)L.p2;
    c.h = (double)L.h;
    c.tol = (double)L.tol;
    c.c0 = L.c0;
    c.c1 = L.c1;
    c.c2 = L.c2;
    c.force = L.force;
    c.trials = (int32_t)L.trials;
    c.prev = last;
    gptr(tp.tape)[slot] = c;
    last = (int)slot;
    return true;
}

// A line inside a cylindrical mapping surface ends on it once the surface is this
// close (reference lengths): its last straight step then errs by about the square of
// this, below the rounding of the compute type's local coordinates.
template <typename T> constexpr double kCylEnd() { return sizeof(T) == 4 ? 1e-5 : 1e-10; }

// A wave refills its idle lanes only once at least this many are idle (or none is
// busy): the refill code runs for the whole wave, so refilling one lane at a time
// would run it on almost every iteration. FP64 steps cost more, so idle lanes cost more
// there and the threshold is lower.
template <typename T> constexpr int refill_min() { return sizeof(T) == 4 ? 24 : 8; }

// TWM: 0 = no twist (narrow records), 1 = twist, 2 = positions only on wide records
// (the FP64 re-trace, which keeps the twist of the first pass); 3 = as 2, held to
// three waves per SIMD (168 VGPRs, about 100 bytes of spills per lane) for calls
// that share the GPU with other maps in flight: its waves then leave room for theirs.
// The FP32 single-job kernel is held to 168 VGPRs so that three waves fit per SIMD
// (the latency of cell fetches is then hidden by more waves), and the FP32 Method II
// kernels to two waves per SIMD (a few bytes of spills; at one wave their lone
// waves took 40% longer than the two-wave form).
// SCH: the integration scheme (Scheme in trace_core.h), the adjoint's forward pass
// (TAPE) included. M2: Method II, the tangent vectors U, V ride along (their
// end values go to the records' uv array).
template <typename T, typename S, int TWM, bool UNI, bool TAPE, int SCH = SCH_RKF45, bool M2 = false>
__global__ __launch_bounds__(256, ((sizeof(T) == 4 && TWM == 1 && UNI && !M2) || TWM == 3) ? 3 : ((sizeof(T) == 4 && M2) ? 2 : 1)) void trace_kernel(const TraceJob *__restrict__ jobs,
                                                    TraceParams tp,
                                                    unsigned long long *__restrict__ counter)
{
    using N = Num<T>;
    constexpr bool TW = TWM == 1;
    // cylindrical mapping surfaces: the multi-job Method I kernels only
    constexpr bool CYLK = !UNI && !M2 && !TAPE;
    // stretched grids: the multi-job kernels, and the adjoint's single-job forward pass
    constexpr bool STRK = !UNI || TAPE;
    const int lane = threadIdx.x & 63;

    // queue size
    int64_t total = tp.static_items;
    if (tp.list) {
        total = (int64_t)(*tp.list_count);
        if (total > tp.list_cap) total = tp.list_cap;
    } else if (!UNI && tp.dynamic_last) {
        total = *tp.total_dev;  // with the rotated-S0 jobs, sized on the device
    }

    // lane state
    int jb = -1;              // job of the active half line, -1 = idle
    bool exhausted = false;
    bool need_load = false;   // the cell changed: fetch its corners before stepping
    bool fresh = false;       // first step of a half line: set h and tol first
    int64_t rec = 0;          // record slot of the active half line
    Lane<T> L{};
    LaneConst<T> K{};
    K.max_steps = tp.max_steps;
    const void *nodes = nullptr;
    if (UNI) {
        const TraceJob &J0 = jobs[0];
        nodes = J0.nodes;
        K.nx = J0.n[0];
        K.ny = J0.n[1];
        K.nz = J0.n[2];
        K.rx = (T)J0.rscale[0];
        K.ry = (T)J0.rscale[1];
        K.rz = (T)J0.rscale[2];
        K.twk = (T)J0.twk;
        K.bnull2 = (T)((double)N::null_rel * (double)(*J0.bmax2));
    }
    // stretched grids (jobs of the multi-job kernels only, which the launcher picks
    // for them): the per-cell scales follow the lane's cell; the length unit is the
    // grid's smallest cell width, found on the device
    bool str = false;
    double dref_s = 0.0;
    if (UNI && TAPE && jobs[0].geo != nullptr) {
        str = true;
        dref_s = jobs[0].geo->dref;
        K.twk = (T)(dref_s * (0.25 / M_PI));
    }
    // cylindrical mapping surfaces (multi-job kernels only, as stretched grids): the
    // lane's job runs inside the cylinder; the state before the trial step (a step
    // that leaves the cylinder is taken again, shorter) and phi = r^2 - R^2 there
    bool cylj = false;
    int sv_c0 = 0, sv_c1 = 0, sv_c2 = 0;
    T sv_p0 = T(0), sv_p1 = T(0), sv_p2 = T(0);
    double sv_tw = 0.0, sv_len = 0.0, cphi = 0.0;
    T cb[3][8], cj[3][8];
    Tan<T> tn;  // Method II
    // Per-XCD queues: the items in 8 contiguous ranges of whole tiles, range x drained
    // first by the workgroups of XCD x (workgroups are dealt to the 8 XCDs in turn),
    // then by any: the lines in flight on one XCD come from one part of the tile order
    // and share more of that XCD's L2. A wave moves to the next range once it has seen
    // its range run out, and is done once it has seen all 8 run out.
    const bool xsplit = !UNI && tp.xcd_ctr != nullptr && !tp.list;
    int xq = (int)(blockIdx.x & 7), xtried = 0;
    const int64_t xr = xsplit ? ((total + 8 * 128 - 1) / (8 * 128)) * 128 : 0;
    unsigned n_trial = 0, n_acc = 0, n_fetch = 0, n_half = 0;
    int acc_half = 0, nck = 0;  // TAPE: accepted steps and checkpoints of the half line
    int last_ck = -1;           // TAPE: pool slot of the last checkpoint

    for (;;) {
        int fin_st = -1, fin_face = -1;  // set when the active half line ends this iteration

        // ---- refill idle lanes: one atomic per wave ------------------------------------
        const bool need = (jb < 0) && !exhausted;
        unsigned long long m = __ballot(need);
        if (m && __popcll(m) < refill_min<T>() && __ballot(jb >= 0) != 0) m = 0;
        if (m) {
            const int cnt = __popcll(m);
            const int leader = __ffsll((long long)m) - 1;
            unsigned long long base = 0;
            int64_t lo = 0, hi = total;
            if (xsplit) {
                lo = (int64_t)xq * xr < total ? (int64_t)xq * xr : total;
                hi = lo + xr < total ? lo + xr : total;
                if (lane == leader) base = atomicAdd(tp.xcd_ctr + 8 * xq, (unsigned long long)cnt);
            } else if (lane == leader) {
                base = atomicAdd(counter, (unsigned long long)cnt);
            }
            base = shfl_u64(base, leader);
            if (xsplit && lo + (int64_t)base + cnt >= hi) {
                xq = (xq + 1) & 7;  // this range has run out
                xtried++;
            }
            if (need) {
                const int rank = __popcll(m & ((1ull << lane) - 1ull));
                const int64_t it = lo + (int64_t)(base + (unsigned long long)rank);
                if (it >= hi) {
                    if (!xsplit || xtried >= 8) exhausted = true;
                } else {
                    int j = 0;
                    int64_t line;
                    bool forward;
                    if (tp.list) {
                        const FixEntry e = gptr(tp.list)[tp.list_rev ? tp.list_cap - 1 - it : it];
                        j = UNI ? 0 : e.job;
                        line = e.line;
                        forward = e.half != 0;
                    } else {
                        // the job whose range of items holds it (the ranges need not
                        // follow the job table's order; rotated-S0 jobs' ranges were set
                        // on the device)
                        if (!UNI)
                            while (j + 1 < tp.njobs &&
                                   !(it >= jobs[j].item_base && it < jobs[j].item_base + 2 * jobs[j].nitems))
                                j++;
                        const TraceJob &J = jobs[j];
                        const int64_t nit = J.nitems;
                        const int64_t local = it - J.item_base;
                        if (J.kind == SEED_PLANE || J.kind == SEED_VOXELS || J.kind == SEED_CYL) {
                            // the forward and backward halves of a tile follow each
                            // other, so long lines of either direction start early
                            forward = ((local >> 6) & 1) == 0;
                            line = line_of_item(J, ((local >> 7) << 6) | (local & 63));
                        } else {
                            forward = local < nit;
                            line = line_of_item(J, forward ? local : local - nit);
                        }
                    }
                    if (line >= 0) {
                        const TraceJob &J = jobs[j];
                        double r[3], nrm[3];
                        seed_of_line<CYLK>(J, line, r, nrm);
                        jb = j;
                        if (!UNI) {
                            nodes = J.nodes;
                            K.nx = J.n[0];
                            K.ny = J.n[1];
                            K.nz = J.n[2];
                            K.rx = (T)J.rscale[0];
                            K.ry = (T)J.rscale[1];
                            K.rz = (T)J.rscale[2];
                            K.twk = (T)J.twk;
                            K.bnull2 = (T)((double)N::null_rel * (double)(*J.bmax2));
                            cylj = J.kind == SEED_CYL;
                            cphi = 0.0;
                            str = J.geo != nullptr;
                            if (str) {
                                dref_s = J.geo->dref;
                                K.twk = (T)(dref_s * (0.25 / M_PI));
                            }
                        }
                        rec = (forward ? J.nlines : 0) + line;
                        L.sgn = forward ? T(1) : T(-1);
                        L.tw = 0.0;
                        L.len = 0.0;
                        L.trials = 0;
                        L.force = -1;
                        acc_half = 0;
                        nck = 0;
                        last_ck = -1;
                        if (STRK && str) {
                            // stretched: the seed's cell by bisection on each axis
                            bool in = !J.geo->bad;
                            for (int a = 0; a < 3; a++) {
                                const FQ_GLOBAL double *x = gptr(J.planes.coord[a]);
                                if (x) in = in && r[a] >= x[0] && r[a] <= x[J.n[a] - 1];
                                else in = in && r[a] >= J.origin[a] &&
                                          r[a] <= J.origin[a] + (J.n[a] - 1) * J.spacing[a];
                            }
                            if (!in) {
                                fin_st = J.geo->bad ? FQ_ST_NONFINITE : FQ_ST_OUTSIDE;
                            } else {
                                double q0, q1, q2;
                                L.c0 = str_cell(J, 0, r[0], q0);
                                L.c1 = str_cell(J, 1, r[1], q1);
                                L.c2 = str_cell(J, 2, r[2], q2);
                                L.p0 = (T)q0;
                                L.p1 = (T)q1;
                                L.p2 = (T)q2;
                                need_load = true;
                                fresh = true;
                            }
                        }
                        if (!STRK || !str) {
                            const double g0 = (r[0] - J.origin[0]) * J.inv_spacing[0],
                                         g1 = (r[1] - J.origin[1]) * J.inv_spacing[1],
                                         g2 = (r[2] - J.origin[2]) * J.inv_spacing[2];
                            if (!(g0 >= 0.0 && g0 <= (double)(K.nx - 1) && g1 >= 0.0 &&
                                  g1 <= (double)(K.ny - 1) && g2 >= 0.0 && g2 <= (double)(K.nz - 1))) {
                                fin_st = FQ_ST_OUTSIDE;
                            } else {
                                L.c0 = min(max((int)floor(g0), 0), K.nx - 2);
                                L.c1 = min(max((int)floor(g1), 0), K.ny - 2);
                                L.c2 = min(max((int)floor(g2), 0), K.nz - 2);
                                L.p0 = (T)(g0 - L.c0);
                                L.p1 = (T)(g1 - L.c1);
                                L.p2 = (T)(g2 - L.c2);
                                need_load = true;
                                fresh = true;
                            }
                        }
                    }
                }
            }
        }

        // ---- fetch the cell (the only load site) ----------------------------------------
        if (jb >= 0 && need_load) {
            load_cell<T, S, TW, TWM != 0>(nodes, K.nx, K.ny, L.c0, L.c1, L.c2, cb, cj);
            need_load = false;
            n_fetch++;
            if (STRK && str) {
                // stretched grid: this cell's widths scale the direction into local
                // coordinates (reference length / width per axis)
                const TraceJob &J = jobs[UNI ? 0 : jb];
                K.rx = (T)(dref_s * gptr(J.iw[0])[L.c0]);
                K.ry = (T)(dref_s * gptr(J.iw[1])[L.c1]);
                K.rz = (T)(dref_s * gptr(J.iw[2])[L.c2]);
            }
            if (fresh) {
                // Eq. step and Eq. tol from the field angle |Bn0/B| at the seed
                fresh = false;
                const TraceJob &J = jobs[UNI ? 0 : jb];
                const float bx = (float)poly<T>(cb[0], L.p0, L.p1, L.p2);
                const float by = (float)poly<T>(cb[1], L.p0, L.p1, L.p2);
                const float bz = (float)poly<T>(cb[2], L.p0, L.p1, L.p2);
                const float b2 = bx * bx + by * by + bz * bz;
                float n0 = (float)J.normal[0], n1 = (float)J.normal[1], n2 = (float)J.normal[2];
                if (CYLK && cylj) {
                    // S0 is the cylinder: its outward normal at the seed
                    n0 = (float)((grid_pos(J, 0, L.c0, (double)L.p0) - J.cyl[0]) / J.cyl[2]);
                    n1 = (float)((grid_pos(J, 1, L.c1, (double)L.p1) - J.cyl[1]) / J.cyl[2]);
                    n2 = 0.0f;
                }
                const float bn = bx * n0 + by * n1 + bz * n2;
                // |Bn0/B| is taken no smaller than 0.05 where S0 is interior (the map
                // rotates S0 perpendicular to B below that), but on a box face, where
                // S0 is the physical S1, the angle itself scales the bound: near a
                // polarity inversion line Bn at the far end is as small as the seed's
                // distance from that line, so the far footpoint must be found to a
                // small fraction of it, which the ang^1.5 of Eq. tol provides
                const bool on_face = (L.c0 == 0 && L.p0 == T(0)) || (L.c0 == K.nx - 2 && L.p0 == T(1)) ||
                                     (L.c1 == 0 && L.p1 == T(0)) || (L.c1 == K.ny - 2 && L.p1 == T(1)) ||
                                     (L.c2 == 0 && L.p2 == T(0)) || (L.c2 == K.nz - 2 && L.p2 == T(1));
                const float amin = on_face ? 1e-9f : 0.05f;
                // Method II's S0 is perpendicular to B: no angle scaling
                float ang = (J.kind == SEED_ROTATED || M2) ? 1.0f : fabsf(bn) * Num<float>::rsq(b2);
                if (!(ang >= amin)) ang = amin;  // also catches NaN
                if (ang > 1.0f) ang = 1.0f;
                L.h = (T)fmaxf((float)tp.step_perp * ang, (float)tp.step_min);
                if (STRK && str) {
                    // stretched grid: the first step in units of the seed cell's width
                    // along B, 1 / |(b_x / dx, b_y / dy, b_z / dz)| (Section 2.3)
                    const float sx = bx * (float)K.rx, sy = by * (float)K.ry, sz = bz * (float)K.rz;
                    const float w2 = sx * sx + sy * sy + sz * sz;
                    if (w2 > 0.0f) L.h = (T)((float)L.h * sqrtf(b2 / w2));
                }
                // a fixed-step scheme keeps its step where RKF45 keeps its bound
                L.tol = SCH != SCH_RKF45 ? L.h : (T)fmax(tp.tol_perp * (double)(ang * sqrtf(ang)), tp.tol_floor);
                if (CYLK && cylj && !((float)L.sgn * bn < 0.0f)) {
                    // heading out of (or along) the cylinder: the half ends at its seed
                    fin_st = 0;
                    fin_face = kFaceCyl;
                }
                if constexpr (M2) {
                    // S0 perpendicular to B at the seed, U and V orthonormal in it:
                    // U = e_a x b / |..| with e_a the axis least aligned with b, V = b x U
                    // (physical units), held in local grid units
                    using N = Num<T>;
                    const T Bx = poly<T>(cb[0], L.p0, L.p1, L.p2), By = poly<T>(cb[1], L.p0, L.p1, L.p2),
                            Bz = poly<T>(cb[2], L.p0, L.p1, L.p2);
                    const T inv = N::rsq(N::fma_(Bx, Bx, N::fma_(By, By, Bz * Bz)));
                    const T b[3] = {Bx * inv, By * inv, Bz * inv};
                    int a = 0;
                    if (fabs(b[1]) < fabs(b[a])) a = 1;
                    if (fabs(b[2]) < fabs(b[a])) a = 2;
                    // e_a x b
                    T u[3] = {a == 0 ? T(0) : (a == 1 ? b[2] : -b[1]),
                              a == 0 ? -b[2] : (a == 1 ? T(0) : b[0]),
                              a == 0 ? b[1] : (a == 1 ? -b[0] : T(0))};
                    const T iu = N::rsq(N::fma_(u[0], u[0], N::fma_(u[1], u[1], u[2] * u[2])));
                    for (int q = 0; q < 3; q++) u[q] *= iu;
                    const T v[3] = {b[1] * u[2] - b[2] * u[1], b[2] * u[0] - b[0] * u[2],
                                    b[0] * u[1] - b[1] * u[0]};
                    for (int q = 0; q < 3; q++) {
                        tn.u[q] = u[q] * (T)J.inv_spacing[q];
                        tn.v[q] = v[q] * (T)J.inv_spacing[q];
                    }
                }
                if (TAPE) {
                    if (store_ckpt<T, TWM, UNI, TAPE>(tp, last_ck, L)) nck++;
                    else fin_st = FQ_ST_MAXSTEPS | FQ_ST_NOTAPE;  // no checkpoint space
                }
            }
        }

        // ---- one trial step -------------------------------------------------------------
        if (jb >= 0 && fin_st < 0) {
            n_trial++;
            const unsigned acc_before = n_acc;
            if (CYLK && cylj) {
                sv_c0 = L.c0, sv_c1 = L.c1, sv_c2 = L.c2;
                sv_p0 = L.p0, sv_p1 = L.p1, sv_p2 = L.p2;
                sv_tw = L.tw, sv_len = L.len;
            }
            lane_iterate<T, TW, NoEvents, SCH, M2>(L, cb, cj, K, fin_st, fin_face, need_load, n_acc,
                                                   NoEvents(), &tn);
            if (CYLK && cylj && fin_st < 0 && n_acc != acc_before) {
                // Inside a cylindrical mapping surface: a step that ends outside it is
                // taken again from its start, shorter (the secant estimate of where phi
                // = r^2 - R^2 changes sign, undershot); near the surface the steps are
                // held short of it, and within kCylEnd reference lengths the line
                // ends on it with one straight step.
                const TraceJob &J = jobs[jb];
                const double dl = str ? dref_s : J.dref;
                const double x = grid_pos(J, 0, L.c0, (double)L.p0), y = grid_pos(J, 1, L.c1, (double)L.p1),
                             z = grid_pos(J, 2, L.c2, (double)L.p2);
                const double dx = x - J.cyl[0], dy = y - J.cyl[1];
                const double phi = dx * dx + dy * dy - J.cyl[2] * J.cyl[2];
                if (phi > 0.0) {
                    const double H = L.len - sv_len;
                    const double tsec = H * (-cphi) / (phi - cphi);
                    if (L.c0 != sv_c0 || L.c1 != sv_c1 || L.c2 != sv_c2) need_load = true;
                    L.c0 = sv_c0, L.c1 = sv_c1, L.c2 = sv_c2;
                    L.p0 = sv_p0, L.p1 = sv_p1, L.p2 = sv_p2;
                    L.tw = sv_tw, L.len = sv_len;
                    L.force = -1;
                    L.h = (T)fmax(fmin(0.9 * tsec, 0.5 * H), (double)N::hmin);
                } else {
                    cphi = phi;
                    const double r[3] = {x, y, z};
                    double B[3];
                    interp64(J.planes, r, B);
                    const double sg = (double)L.sgn / sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
                    const double ux = sg * B[0], uy = sg * B[1], uz = sg * B[2];
                    const double b1 = dx * ux + dy * uy;  // half of d phi / ds
                    if (b1 > 0.0) {
                        const double est = -phi / (2.0 * b1);
                        if (est <= kCylEnd<T>() * dl) {
                            // phi + 2 b1 t + (ux^2 + uy^2) t^2 = 0, its root t >= 0
                            const double t = -phi / (b1 + sqrt(b1 * b1 - (ux * ux + uy * uy) * phi));
                            L.p0 += (T)(t * ux * inv_width(J, 0, L.c0));
                            L.p1 += (T)(t * uy * inv_width(J, 1, L.c1));
                            L.p2 += (T)(t * uz * inv_width(J, 2, L.c2));
                            L.len += t / dl;
                            fin_st = 0;
                            fin_face = kFaceCyl;
                        } else if ((double)L.h * dl > 0.9 * est) {
                            L.h = (T)(0.9 * est / dl);
                        }
                    }
                }
            }
            if (TAPE && n_acc != acc_before) {
                acc_half++;
                if (fin_st < 0 && acc_half % tp.seg == 0) {
                    if (store_ckpt<T, TWM, UNI, TAPE>(tp, last_ck, L)) {
                        nck++;
                    } else {
                        fin_st = FQ_ST_MAXSTEPS | FQ_ST_NOTAPE;  // no checkpoint space
                        fin_face = -1;
                    }
                }
            }
        }

        // ---- write the record of a finished half line -----------------------------------
        if (jb >= 0 && fin_st >= 0) {
            const TraceJob &J = jobs[UNI ? 0 : jb];
            const bool bad = (fin_st & (FQ_ST_OUTSIDE | FQ_ST_NULLB | FQ_ST_MAXSTEPS | FQ_ST_NONFINITE)) != 0;
            double e0 = NAN, e1 = NAN, e2 = NAN;
            if (!bad && L.len == 0.0) {
                // no step taken (a seed on a box face heading out of the box): the
                // half line ends exactly at its seed, not at the seed's position as
                // rounded into local coordinates of the compute type
                double r[3], nrm[3];
                seed_of_line<CYLK>(J, rec >= J.nlines ? rec - J.nlines : rec, r, nrm);
                e0 = r[0];
                e1 = r[1];
                e2 = r[2];
            } else if (!bad && STRK && str) {
                e0 = grid_pos(J, 0, L.c0, (double)L.p0);
                e1 = grid_pos(J, 1, L.c1, (double)L.p1);
                e2 = grid_pos(J, 2, L.c2, (double)L.p2);
            } else if (!bad) {
                e0 = J.origin[0] + ((double)L.c0 + (double)L.p0) * J.spacing[0];
                e1 = J.origin[1] + ((double)L.c1 + (double)L.p1) * J.spacing[1];
                e2 = J.origin[2] + ((double)L.c2 + (double)L.p2) * J.spacing[2];
            }
            FQ_GLOBAL double *ge = gptr(J.rec.end);
            ge[3 * rec + 0] = e0;
            ge[3 * rec + 1] = e1;
            ge[3 * rec + 2] = e2;
            if (TWM != 2 && TWM != 3) gptr(J.rec.tw)[rec] = bad ? NAN : (TW ? L.tw : NAN);
            gptr(J.rec.len)[rec] = bad ? NAN : L.len * ((STRK && str) ? dref_s : J.dref);
            gptr(J.rec.face)[rec] = bad ? (int8_t)-1 : (int8_t)fin_face;
            gptr(J.rec.st)[rec] = (uint16_t)fin_st;
            if constexpr (M2) {
                FQ_GLOBAL double *uv = gptr(J.rec.uv) + 6 * rec;
                for (int q = 0; q < 3; q++) {
                    uv[q] = bad ? NAN : (double)tn.u[q] * J.spacing[q];
                    uv[3 + q] = bad ? NAN : (double)tn.v[q] * J.spacing[q];
                }
            }
            if (TAPE) {
                // an interior seed plane's rotated-S0 job keeps its records after the
                // main job's
                const int64_t trec = rec + (jb > 0 ? tp.tape_base1 : 0);
                gptr(tp.tape_last)[trec] = last_ck;
                gptr(tp.tape_n)[trec] = nck;
                gptr(tp.tape_acc)[trec] = acc_half;
            }
            jb = -1;
            need_load = false;
            n_half++;
        }

        if (__ballot(jb >= 0) == 0 && __ballot(!exhausted) == 0) break;
    }
    if (tp.stats) {
        const bool fix = tp.list != nullptr;
        unsigned long long v[5] = {n_trial, n_acc, n_fetch, fix ? 0u : n_half, fix ? n_half : 0u};
#pragma unroll
        for (int q = 0; q < 5; q++) {
            unsigned long long x = v[q];
            for (int off = 32; off > 0; off >>= 1) {
                unsigned lo = __shfl_xor((unsigned)x, off), hi = __shfl_xor((unsigned)(x >> 32), off);
                x += ((unsigned long long)hi << 32) | lo;
            }
            if (lane == 0 && x) atomicAdd(tp.stats + q, x);
        }
    }
}

// Lines whose field is nearly tangent to S0 at the seed, or half lines whose field
// is nearly tangent to the face they end on, turn FP32 rounding into large footpoint
// errors (a height error d of a line meeting a plane at angle a moves its crossing
// by d/a); those half lines, and any the FP32 pass could not finish, are listed for
// the FP64 pass. So are both halves of a line whose map point (qmap, the Q the FP32
// pass gives: one point per line of a plane or voxel job; for the four lines of a
// rotated-S0 entry, the entry's point) has Q above qthr: the map stretches a line's
// rounding error by about sqrt(Q). Half lines the FP32 pass could not finish have no
// twist either: with split they go to the second list (from the top of the array
// down), which is traced with the twist integrand after a positions-only pass over
// the first; without it they join the first list. seed_check: the seed's angle with
// S0 is tested (Method II's S0 is perpendicular to B and has no such test).
__global__ void graze_kernel(const TraceJob *__restrict__ jobs, int job, double thr,
                             const double *__restrict__ qmap, double qthr,
                             FixEntry *__restrict__ list, uint32_t *__restrict__ count,
                             uint32_t *__restrict__ count_tw, int64_t cap, int split, int seed_check)
{
    const TraceJob &J = jobs[job];
    const int64_t nl = live_lines(J);
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < nl;
         l += (int64_t)gridDim.x * blockDim.x) {
        const int64_t hb = l, hf = J.nlines + l;
        const uint16_t sb = J.rec.st[hb], sf = J.rec.st[hf];
        const uint16_t hard = FQ_ST_OUTSIDE | FQ_ST_NULLB | FQ_ST_NONFINITE;
        if ((sb | sf) & hard) continue;
        // a half line is traced again if the FP32 pass could not finish it, if the
        // seed is grazing (both halves then stepped at the tolerance floor), or if
        // its own end is grazing (the footpoint error is amplified at its own end only)
        bool seed_graze = false;
        if (seed_check && J.kind != SEED_ROTATED) {
            double r[3], nrm[3], B[3];
            seed_of_line(J, l, r, nrm);
            interp64(J.planes, r, B);
            const double bm = sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
            const double bn = B[0] * nrm[0] + B[1] * nrm[1] + B[2] * nrm[2];
            seed_graze = !(fabs(bn) >= thr * bm);
        }
        if (qmap) {
            if ((J.kind == SEED_PLANE || J.kind == SEED_VOXELS || J.kind == SEED_CYL) && l < J.nlines &&
                qmap[l] > qthr)
                seed_graze = true;
            if (J.kind == SEED_ROTATED && qmap[J.rot[l >> 2].point] > qthr) seed_graze = true;
        }
        for (int h = 0; h < 2; h++) {
            const int64_t q = h ? hf : hb;
            if (J.rec.len[q] == 0.0) continue;  // ends at its seed: nothing to improve
            const bool unfinished = (J.rec.st[q] & FQ_ST_MAXSTEPS) != 0;
            bool redo = seed_graze;
            const int face = J.rec.face[q];
            if (!redo && !unfinished && face >= 0) {
                const double e[3] = {J.rec.end[3 * q], J.rec.end[3 * q + 1], J.rec.end[3 * q + 2]};
                double B[3];
                interp64(J.planes, e, B);
                const double bm = sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
                double bnf;
                if (face == kFaceCyl) {
                    // an end on a cylindrical mapping surface: along its outward normal
                    const double dx = e[0] - J.cyl[0], dy = e[1] - J.cyl[1];
                    bnf = (B[0] * dx + B[1] * dy) / sqrt(dx * dx + dy * dy);
                } else {
                    bnf = face == 0 || face == 1 ? B[0] : (face == 2 || face == 3 ? B[1] : B[2]);
                }
                redo = !(fabs(bnf) >= thr * bm);
            }
            if (unfinished && split) {
                const uint32_t k = atomicAdd(count_tw, 1u);
                if ((int64_t)k < cap) list[cap - 1 - k] = FixEntry{job, h, l};
            } else if (redo || unfinished) {
                const uint32_t slot = atomicAdd(count, 1u);
                if ((int64_t)slot < cap) list[slot] = FixEntry{job, h, l};
            }
        }
    }
}

template <typename T, typename S, bool UNI, int SCH>
const void *kernel_of_s(int twm)
{
    if constexpr (sizeof(T) == 8)
        if (twm == 3) return (const void *)trace_kernel<T, S, 3, UNI, false, SCH>;
    return twm == 1 ? (const void *)trace_kernel<T, S, 1, UNI, false, SCH>
                    : twm == 2 ? (const void *)trace_kernel<T, S, 2, UNI, false, SCH>
                               : (const void *)trace_kernel<T, S, 0, UNI, false, SCH>;
}

template <typename T, typename S, bool UNI>
const void *kernel_of(int twm, int sch, int method)
{
    if (method == FQ_METHOD_II)
        return twm == 1 ? (const void *)trace_kernel<T, S, 1, UNI, false, SCH_RKF45, true>
                        : (const void *)trace_kernel<T, S, 0, UNI, false, SCH_RKF45, true>;
    return sch == SCH_RK4 ? kernel_of_s<T, S, UNI, SCH_RK4>(twm)
                          : sch == SCH_RK4_38 ? kernel_of_s<T, S, UNI, SCH_RK4_38>(twm)
                                              : kernel_of_s<T, S, UNI, SCH_RKF45>(twm);
}

template <typename T, typename S, bool UNI, bool TAPE, int SCH>
void launch_tss(int twm, dim3 grid, dim3 blk, hipStream_t s, const TraceJob *jobs,
                const TraceParams &tp, unsigned long long *counter)
{
    if constexpr (sizeof(T) == 8 && !TAPE)
        if (twm == 3) {
            hipLaunchKernelGGL((trace_kernel<T, S, 3, UNI, false, SCH>), grid, blk, 0, s, jobs, tp, counter);
            return;
        }
    if (twm == 1) hipLaunchKernelGGL((trace_kernel<T, S, 1, UNI, TAPE, SCH>), grid, blk, 0, s, jobs, tp, counter);
    else if (twm == 2 && !TAPE) hipLaunchKernelGGL((trace_kernel<T, S, 2, UNI, false, SCH>), grid, blk, 0, s, jobs, tp, counter);
    else hipLaunchKernelGGL((trace_kernel<T, S, 0, UNI, TAPE, SCH>), grid, blk, 0, s, jobs, tp, counter);
}

template <typename T, typename S, bool UNI>
void launch_m2(int twm, dim3 grid, dim3 blk, hipStream_t s, const TraceJob *jobs,
               const TraceParams &tp, unsigned long long *counter)
{
    if (twm == 1) hipLaunchKernelGGL((trace_kernel<T, S, 1, UNI, false, SCH_RKF45, true>), grid, blk, 0, s, jobs, tp, counter);
    else hipLaunchKernelGGL((trace_kernel<T, S, 0, UNI, false, SCH_RKF45, true>), grid, blk, 0, s, jobs, tp, counter);
}

template <typename T, typename S, bool UNI, bool TAPE>
void launch_ts(int twm, dim3 grid, dim3 blk, hipStream_t s, const TraceJob *jobs,
               const TraceParams &tp, unsigned long long *counter)
{
    if (!TAPE && tp.method == FQ_METHOD_II) launch_m2<T, S, UNI>(twm, grid, blk, s, jobs, tp, counter);
    else if (tp.scheme == SCH_RKF45) launch_tss<T, S, UNI, TAPE, SCH_RKF45>(twm, grid, blk, s, jobs, tp, counter);
    else if (tp.scheme == SCH_RK4) launch_tss<T, S, UNI, TAPE, SCH_RK4>(twm, grid, blk, s, jobs, tp, counter);
    else launch_tss<T, S, UNI, TAPE, SCH_RK4_38>(twm, grid, blk, s, jobs, tp, counter);
}

__global__ void fill_counts_kernel(uint32_t *counts)
{
    counts[threadIdx.x] = 0u;
}

// Tile order of a plane job: long lines start early, so the last ones to finish are
// short. A tile's key is the length of the longest of ten coarse half lines: its four
// corner seeds and a central one, traced both ways with Heun steps of four grid
// spacings (at most 256), in FP32 on the tracer's own node records (B in the first
// four values of a record of type R; 8-wide records when WIDE). Half lines are the
// queue's items, so the longest half decides when a tile's work ends; the key is the
// step count, and tiles are placed longest first (the order inside a key does not
// matter: every line's result is independent of when it is traced).
constexpr int kCoarseCells = 4, kCoarseSteps = 256;

// B at grid coordinates g (clamped into the grid) from the node records.
template <typename R, bool WIDE>
__device__ __forceinline__ void coarse_field(const typename V4<R>::t *__restrict__ A, const int n[3],
                                             const float g[3], float B[3])
{
    int c[3];
    float t[3];
    for (int a = 0; a < 3; a++) {
        const float x = fminf(fmaxf(g[a], 0.0f), (float)(n[a] - 1));
        int ci = (int)floorf(x);
        ci = ci > n[a] - 2 ? n[a] - 2 : ci;
        c[a] = ci;
        t[a] = x - (float)ci;
    }
    const int64_t sy = n[0], sz = (int64_t)n[0] * n[1];
    const int64_t base = (int64_t)c[2] * sz + (int64_t)c[1] * sy + c[0];
    B[0] = B[1] = B[2] = 0.0f;
#pragma unroll
    for (int q = 0; q < 8; q++) {
        const int ix = q & 1, iy = (q >> 1) & 1, iz = (q >> 2) & 1;
        const float w = (ix ? t[0] : 1.0f - t[0]) * (iy ? t[1] : 1.0f - t[1]) * (iz ? t[2] : 1.0f - t[2]);
        const int64_t o = base + ix + iy * sy + iz * sz;
        const typename V4<R>::t v = A[WIDE ? 2 * o : o];
        B[0] = fmaf(w, (float)v.x, B[0]);
        B[1] = fmaf(w, (float)v.y, B[1]);
        B[2] = fmaf(w, (float)v.z, B[2]);
    }
}

template <typename R, bool WIDE>
__global__ void tile_len_kernel(TraceJob J, int32_t *__restrict__ len)
{
    const typename V4<R>::t *A = gptr((const typename V4<R>::t *)J.nodes);
    const int64_t ntiles = J.tiles[0] * J.tiles[1];
    // stretched grids: grid coordinates run through the cells at their own widths,
    // so a coarse step's size in grid units follows the cell it starts in
    const bool str = J.geo != nullptr;
    const double dmin = str ? J.geo->dref : fmin(J.spacing[0], fmin(J.spacing[1], J.spacing[2]));
    const int n[3] = {J.n[0], J.n[1], J.n[2]};
    float hs[3];  // a coarse step along a unit direction, in grid units per axis
    for (int a = 0; a < 3; a++) hs[a] = (float)(kCoarseCells * dmin / J.spacing[a]);
    auto step_of = [&](int a, float ga) -> float {
        if (!str) return hs[a];
        const int c = min(max((int)floorf(ga), 0), n[a] - 2);
        return (float)(kCoarseCells * dmin * J.iw[a][c]);
    };
    const int sw[5] = {0, 7, 56, 63, 36};
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < 10 * ntiles;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = k / 10;
        const int q = (int)(k - 10 * t);
        const float sgn = (q & 1) ? -1.0f : 1.0f;
        const int64_t ty = t / J.tiles[0], tx = t - ty * J.tiles[0];
        const int w = sw[q >> 1];
        int64_t i = tx * 8 + (w & 7), j = ty * 8 + (w >> 3);
        i = i < J.dims[0] ? i : J.dims[0] - 1;
        j = j < J.dims[1] ? j : J.dims[1] - 1;
        float g[3];
        bool inside = true;
        for (int a = 0; a < 3; a++) {
            const double r = J.s_origin[a] + (double)i * J.s_a[a] + (double)j * J.s_b[a];
            if (str && J.planes.coord[a]) {
                const double *x = J.planes.coord[a];
                inside = inside && r >= x[0] && r <= x[n[a] - 1];
                double p;
                const int c = str_cell(J, a, r, p);
                g[a] = (float)((double)c + p);
                continue;
            }
            g[a] = (float)((r - J.origin[a]) * J.inv_spacing[a]);
            inside = inside && g[a] >= 0.0f && g[a] <= (float)(n[a] - 1);
        }
        int m = 0;
        if (inside) {
            for (; m < kCoarseSteps; m++) {
                float B[3], gm[3], B2[3];
                coarse_field<R, WIDE>(A, n, g, B);
                const float bm = sqrtf(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
                if (!(bm > 0.0f) || !isfinite(bm)) break;
                for (int a = 0; a < 3; a++) gm[a] = g[a] + 0.5f * sgn * step_of(a, g[a]) * B[a] / bm;
                coarse_field<R, WIDE>(A, n, gm, B2);
                const float bm2 = sqrtf(B2[0] * B2[0] + B2[1] * B2[1] + B2[2] * B2[2]);
                if (!(bm2 > 0.0f) || !isfinite(bm2)) break;
                bool in = true;
                for (int a = 0; a < 3; a++) {
                    g[a] += sgn * step_of(a, gm[a]) * B2[a] / bm2;
                    in = in && g[a] >= 0.0f && g[a] <= (float)(n[a] - 1);
                }
                if (!in) break;
            }
        }
        atomicMax(len + t, m);
    }
}

// Tile order of a 3-D (voxel) job: a voxel map's lines sweep the whole cube, whose
// node records do not fit the caches, so the tiles whose lines run together should be
// traced together. Lines that share a footpoint are one flux tube: a tile's key is
// where the coarse backward line from its central voxel leaves the box (Heun steps
// of four grid spacings, at most 1024), a bin of that face, the bins of each face in
// a serpentine order so that neighbouring keys are neighbouring bins: 224 x 224 bins
// on the bottom face (z low, where most lines of a solar cube end), 50 x 60 on each
// other face, and the last key (65535) for a line that does not leave. The tiles are
// then placed by a counting sort over the 65536 keys (in any order inside a key).
constexpr int kFootSteps = 1024;
constexpr int kFootKeys = 65536;

__device__ __forceinline__ int serp(float u, float v, int nu, int nv)
{
    const int iu = min(max((int)(u * (float)nu), 0), nu - 1);
    const int iv = min(max((int)(v * (float)nv), 0), nv - 1);
    return iv * nu + ((iv & 1) ? nu - 1 - iu : iu);
}

template <typename R, bool WIDE>
__global__ void tile_foot_kernel(TraceJob J, int32_t *__restrict__ key)
{
    const typename V4<R>::t *A = gptr((const typename V4<R>::t *)J.nodes);
    const int64_t ntiles = J.tiles[0] * J.tiles[1] * J.tiles[2];
    const bool str = J.geo != nullptr;
    const double dmin = str ? J.geo->dref : fmin(J.spacing[0], fmin(J.spacing[1], J.spacing[2]));
    const int n[3] = {J.n[0], J.n[1], J.n[2]};
    float hs[3];
    for (int a = 0; a < 3; a++) hs[a] = (float)(kCoarseCells * dmin / J.spacing[a]);
    auto step_of = [&](int a, float ga) -> float {
        if (!str) return hs[a];
        const int c = min(max((int)floorf(ga), 0), n[a] - 2);
        return (float)(kCoarseCells * dmin * J.iw[a][c]);
    };
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t tz = t / (J.tiles[0] * J.tiles[1]);
        const int64_t rem = t - tz * J.tiles[0] * J.tiles[1];
        const int64_t ty = rem / J.tiles[0], tx = rem - ty * J.tiles[0];
        const int64_t iv[3] = {min(tx * 4 + 2, J.dims[0] - 1), min(ty * 4 + 2, J.dims[1] - 1),
                               min(tz * 4 + 2, J.dims[2] - 1)};
        const double sp[3] = {J.s_a[0], J.s_b[1], J.s_c[2]};
        float g[3];
        bool inside = true;
        for (int a = 0; a < 3; a++) {
            const double r = J.s_origin[a] + (double)iv[a] * sp[a];
            if (str && J.planes.coord[a]) {
                const double *x = J.planes.coord[a];
                inside = inside && r >= x[0] && r <= x[n[a] - 1];
                double p;
                const int c = str_cell(J, a, r, p);
                g[a] = (float)((double)c + p);
                continue;
            }
            g[a] = (float)((r - J.origin[a]) * J.inv_spacing[a]);
            inside = inside && g[a] >= 0.0f && g[a] <= (float)(n[a] - 1);
        }
        int k = kFootKeys - 1;
        if (inside) {
            bool left = false;
            for (int m = 0; m < kFootSteps && !left; m++) {
                float B[3], gm[3], B2[3];
                coarse_field<R, WIDE>(A, n, g, B);
                const float bm = sqrtf(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
                if (!(bm > 0.0f) || !isfinite(bm)) break;
                for (int a = 0; a < 3; a++) gm[a] = g[a] - 0.5f * step_of(a, g[a]) * B[a] / bm;
                coarse_field<R, WIDE>(A, n, gm, B2);
                const float bm2 = sqrtf(B2[0] * B2[0] + B2[1] * B2[1] + B2[2] * B2[2]);
                if (!(bm2 > 0.0f) || !isfinite(bm2)) break;
                for (int a = 0; a < 3; a++) {
                    g[a] -= step_of(a, gm[a]) * B2[a] / bm2;
                    left = left || g[a] < 0.0f || g[a] > (float)(n[a] - 1);
                }
            }
            if (left) {
                // the face it left by: the farthest out (grid units)
                int f = 0;
                float out = -1.0f;
                for (int a = 0; a < 3; a++) {
                    const float lo = -g[a], hi = g[a] - (float)(n[a] - 1);
                    if (lo > out) out = lo, f = 2 * a;
                    if (hi > out) out = hi, f = 2 * a + 1;
                }
                const int a = f >> 1, b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
                const float u = g[b] / (float)(n[b] - 1), v = g[c] / (float)(n[c] - 1);
                if (f == 4) k = serp(u, v, 224, 224);
                else k = 224 * 224 + 3000 * (f < 4 ? f : 4) + serp(u, v, 50, 60);
            }
        }
        key[t] = k;
    }
}

// Key -> bucket, longest first (bucket 0), and the bucket counts for the placement
// (a block histogram in LDS first: many tiles share a bucket). Blocks of 256.
__global__ void tile_key_kernel(int64_t ntiles, int32_t *__restrict__ bucket,
                                uint32_t *__restrict__ counts)
{
    __shared__ uint32_t hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t n = bucket[t];
        const int b = 255 - (n < 0 ? 0 : (n > 255 ? 255 : n));
        bucket[t] = b;
        atomicAdd(hist + b, 1u);
    }
    __syncthreads();
    if (hist[threadIdx.x]) atomicAdd(counts + threadIdx.x, hist[threadIdx.x]);
}

__global__ void tile_scan_kernel(uint32_t *counts)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        uint32_t acc = 0;
        for (int b = 0; b < 256; b++) {
            const uint32_t c = counts[b];
            counts[b] = acc;
            acc += c;
        }
    }
}

// Each block ranks its tiles inside their buckets in LDS and takes one range per
// bucket from the global offsets. Blocks of 256; every thread runs the same number
// of iterations (the barriers are uniform).
__global__ void tile_place_kernel(int64_t ntiles, const int32_t *__restrict__ bucket,
                                  uint32_t *__restrict__ offsets, int32_t *__restrict__ order)
{
    __shared__ uint32_t hist[256], base[256];
    for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x; t0 < ntiles;
         t0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = t0 + threadIdx.x;
        hist[threadIdx.x] = 0;
        __syncthreads();
        const int b = t < ntiles ? bucket[t] : -1;
        const uint32_t r = b >= 0 ? atomicAdd(hist + b, 1u) : 0u;
        __syncthreads();
        if (hist[threadIdx.x]) base[threadIdx.x] = atomicAdd(offsets + threadIdx.x, hist[threadIdx.x]);
        __syncthreads();
        if (b >= 0) order[base[b] + r] = (int32_t)t;
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_tile_order(const TraceJob &J, int prec, int want_tw, int32_t *bucket,
                             uint32_t *counts, int32_t *order, hipStream_t s)
{
    const int64_t ntiles = J.tiles[0] * J.tiles[1];
    hipError_t e = launch_fill_u32((uint32_t *)bucket, ntiles, 0u, s);
    if (e != hipSuccess) return e;
    int64_t bl = (10 * ntiles + 255) / 256;
    if (bl > 65536) bl = 65536;
    // the node records the prep pass wrote: FP64 values for the all-FP64 form
    if (prec == FQ_PREC_F64) {
        if (want_tw) hipLaunchKernelGGL((tile_len_kernel<double, true>), dim3((unsigned)bl), dim3(256), 0, s, J, bucket);
        else hipLaunchKernelGGL((tile_len_kernel<double, false>), dim3((unsigned)bl), dim3(256), 0, s, J, bucket);
    } else {
        if (want_tw) hipLaunchKernelGGL((tile_len_kernel<float, true>), dim3((unsigned)bl), dim3(256), 0, s, J, bucket);
        else hipLaunchKernelGGL((tile_len_kernel<float, false>), dim3((unsigned)bl), dim3(256), 0, s, J, bucket);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_bucket_order(ntiles, bucket, counts, order, s);
}

namespace {
// The counting sort of voxel tiles by key: counts per key, their exclusive scan (one
// block), and the placement (a key's cursor taken with an atomic: tiles of one key
// land in any order, which only changes when each is traced).
__global__ void foot_count_kernel(int64_t n, const int32_t *__restrict__ key, uint32_t *counts)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(counts + key[t], 1u);
}

__global__ __launch_bounds__(1024) void foot_scan_kernel(uint32_t *counts)
{
    constexpr int per = kFootKeys / 1024;
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    uint32_t sum = 0;
    for (int i = 0; i < per; i++) sum += counts[t * per + i];
    part[t] = sum;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const uint32_t v = t >= d ? part[t - d] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t acc = part[t] - sum;
    for (int i = 0; i < per; i++) {
        const uint32_t c = counts[t * per + i];
        counts[t * per + i] = acc;
        acc += c;
    }
}

__global__ void foot_place_kernel(int64_t n, const int32_t *__restrict__ key, uint32_t *cursor,
                                  int32_t *__restrict__ order)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        order[atomicAdd(cursor + key[t], 1u)] = (int32_t)t;
}
}  // namespace

hipError_t launch_voxel_order(const TraceJob &J, int prec, int want_tw, int32_t *key,
                              uint32_t *counts, int32_t *order, hipStream_t s)
{
    const int64_t ntiles = J.tiles[0] * J.tiles[1] * J.tiles[2];
    int64_t bl = (ntiles + 255) / 256;
    if (bl > 65536) bl = 65536;
    hipError_t e = launch_fill_u32(counts, kFootKeys, 0u, s);
    if (e != hipSuccess) return e;
    if (prec == FQ_PREC_F64) {
        if (want_tw) hipLaunchKernelGGL((tile_foot_kernel<double, true>), dim3((unsigned)bl), dim3(256), 0, s, J, key);
        else hipLaunchKernelGGL((tile_foot_kernel<double, false>), dim3((unsigned)bl), dim3(256), 0, s, J, key);
    } else {
        if (want_tw) hipLaunchKernelGGL((tile_foot_kernel<float, true>), dim3((unsigned)bl), dim3(256), 0, s, J, key);
        else hipLaunchKernelGGL((tile_foot_kernel<float, false>), dim3((unsigned)bl), dim3(256), 0, s, J, key);
    }
    hipLaunchKernelGGL(foot_count_kernel, dim3((unsigned)bl), dim3(256), 0, s, ntiles, key, counts);
    hipLaunchKernelGGL(foot_scan_kernel, dim3(1), dim3(1024), 0, s, counts);
    hipLaunchKernelGGL(foot_place_kernel, dim3((unsigned)bl), dim3(256), 0, s, ntiles, key, counts, order);
    return hipGetLastError();
}

hipError_t launch_bucket_order(int64_t n, int32_t *key, uint32_t *counts, int32_t *order,
                               hipStream_t s)
{
    int64_t b = (n + 255) / 256;
    if (b < 1) b = 1;
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(fill_counts_kernel, dim3(1), dim3(256), 0, s, counts);
    hipLaunchKernelGGL(tile_key_kernel, dim3((unsigned)b), dim3(256), 0, s, n, key, counts);
    hipLaunchKernelGGL(tile_scan_kernel, dim3(1), dim3(64), 0, s, counts);
    hipLaunchKernelGGL(tile_place_kernel, dim3((unsigned)b), dim3(256), 0, s, n, key, counts, order);
    return hipGetLastError();
}

hipError_t launch_trace(int prec, int store, int twm, const TraceJob *jobs_dev,
                        const TraceParams &tp, unsigned long long *counter, int block,
                        int waves_per_cu, hipStream_t s)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) ncu = 0;
    if (ncu <= 0) ncu = 256;
    if (block <= 0) block = 256;
    const bool f64 = prec == FQ_PREC_F64, s64 = store == FQ_DT_F64;
    if (!f64 && s64) return hipErrorInvalidValue;  // FP32 arithmetic reads FP32 records only
    // stretched grids take the multi-job kernels, which carry their per-cell scales
    const bool uni = tp.njobs == 1 && !tp.dynamic_last && !tp.stretched && !tp.cyl;
    if (tp.scheme < SCH_RKF45 || tp.scheme > SCH_RK4_38) return hipErrorInvalidValue;
    if (tp.tape) {
        // the adjoint's forward pass, Method I, no FP64 re-trace list; FP64 on FP64
        // records, or the FP32 pass of the F32X form. One job (the single-job kernels,
        // which carry the stretched-grid lane state for it), or a seed plane and its
        // rotated-S0 job (the multi-job kernels, RKF45).
        const bool one = tp.njobs == 1 && !tp.dynamic_last;
        const bool two = tp.njobs == 2 && tp.dynamic_last && tp.scheme == SCH_RKF45;
        if (!(one || two) || tp.cyl || tp.list || tp.seg < 1 || tp.method != FQ_METHOD_I || f64 != s64)
            return hipErrorInvalidValue;
        const dim3 grid((unsigned)(2 * ncu)), blk(256);
        if (one) {
            if (s64) launch_ts<double, double, true, true>(twm, grid, blk, s, jobs_dev, tp, counter);
            else launch_ts<float, float, true, true>(twm, grid, blk, s, jobs_dev, tp, counter);
        } else if (s64) {
            launch_tss<double, double, false, true, SCH_RKF45>(twm, grid, blk, s, jobs_dev, tp, counter);
        } else {
            launch_tss<float, float, false, true, SCH_RKF45>(twm, grid, blk, s, jobs_dev, tp, counter);
        }
        return hipGetLastError();
    }
    const void *fn;
    const int sch = tp.scheme, mt = tp.method;
    if (mt == FQ_METHOD_II && (sch != SCH_RKF45 || twm == 2 || twm == 3)) return hipErrorInvalidValue;
    if (twm == 3 && !f64) return hipErrorInvalidValue;
    if (!f64) fn = uni ? kernel_of<float, float, true>(twm, sch, mt) : kernel_of<float, float, false>(twm, sch, mt);
    else if (s64) fn = uni ? kernel_of<double, double, true>(twm, sch, mt) : kernel_of<double, double, false>(twm, sch, mt);
    else fn = uni ? kernel_of<double, float, true>(twm, sch, mt) : kernel_of<double, float, false>(twm, sch, mt);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, 0) != hipSuccess) per_cu = 0;
    if (per_cu <= 0) per_cu = 1;
    if (waves_per_cu > 0) {
        int want = (waves_per_cu * 64 + block - 1) / block;
        if (want < per_cu) per_cu = want;
        if (per_cu < 1) per_cu = 1;
    }
    dim3 grid((unsigned)(per_cu * ncu)), blk((unsigned)block);
    if (!f64) {
        if (uni) launch_ts<float, float, true, false>(twm, grid, blk, s, jobs_dev, tp, counter);
        else launch_ts<float, float, false, false>(twm, grid, blk, s, jobs_dev, tp, counter);
    } else if (s64) {
        if (uni) launch_ts<double, double, true, false>(twm, grid, blk, s, jobs_dev, tp, counter);
        else launch_ts<double, double, false, false>(twm, grid, blk, s, jobs_dev, tp, counter);
    } else {
        if (uni) launch_ts<double, float, true, false>(twm, grid, blk, s, jobs_dev, tp, counter);
        else launch_ts<double, float, false, false>(twm, grid, blk, s, jobs_dev, tp, counter);
    }
    return hipGetLastError();
}

namespace {
__global__ void rot_ranges_kernel(TraceJob *jobs, int first, int n, int64_t base, int64_t *total)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int k = first; k < first + n; k++) {
        TraceJob &J = jobs[k];
        const int64_t lines = live_lines(J);
        J.item_base = base;
        J.nitems = ((lines + 63) / 64) * 64;
        base += 2 * J.nitems;
    }
    *total = base;
}
}  // namespace

hipError_t launch_rot_ranges(TraceJob *jobs_dev, int first, int n, int64_t base, int64_t *total,
                             hipStream_t s)
{
    hipLaunchKernelGGL(rot_ranges_kernel, dim3(1), dim3(64), 0, s, jobs_dev, first, n, base, total);
    return hipGetLastError();
}

namespace {
// The FP64 pass's list ordered longest first (by the FP32 pass's length of each half
// line, in cells of the smallest spacing, 4 cells per key; a key per 256): a wave then
// takes lines of like length and frees its SIMD slot when they end, instead of
// holding it for one long line among short ones. Only the list's own entries are
// keyed (the count is on the device); the placement is tile_place_kernel's.
__global__ void fix_key_kernel(const TraceJob *__restrict__ jobs, const FixEntry *__restrict__ list,
                               const uint32_t *__restrict__ count, int64_t cap,
                               int32_t *__restrict__ key, uint32_t *__restrict__ counts)
{
    __shared__ uint32_t hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const int64_t n = (int64_t)*count < cap ? (int64_t)*count : cap;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const FixEntry e = list[t];
        const TraceJob &J = jobs[e.job];
        const double len = J.rec.len[e.half ? J.nlines + e.line : e.line];
        double d = J.spacing[0];
        if (J.spacing[1] < d) d = J.spacing[1];
        if (J.spacing[2] < d) d = J.spacing[2];
        const double c = len / (4.0 * d);
        const int k = !(c > 0.0) ? 0 : (c >= 255.0 ? 255 : (int)c);
        const int b = 255 - k;
        key[t] = b;
        atomicAdd(hist + b, 1u);
    }
    __syncthreads();
    if (hist[threadIdx.x]) atomicAdd(counts + threadIdx.x, hist[threadIdx.x]);
}

__global__ void fix_place_kernel(const FixEntry *__restrict__ list, const uint32_t *__restrict__ count,
                                 int64_t cap, const int32_t *__restrict__ key,
                                 uint32_t *__restrict__ offsets, FixEntry *__restrict__ out)
{
    __shared__ uint32_t hist[256], base[256];
    const int64_t n = (int64_t)*count < cap ? (int64_t)*count : cap;
    for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x; t0 < n; t0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = t0 + threadIdx.x;
        hist[threadIdx.x] = 0;
        __syncthreads();
        const int b = t < n ? key[t] : -1;
        const uint32_t r = b >= 0 ? atomicAdd(hist + b, 1u) : 0u;
        __syncthreads();
        if (hist[threadIdx.x]) base[threadIdx.x] = atomicAdd(offsets + threadIdx.x, hist[threadIdx.x]);
        __syncthreads();
        if (b >= 0) out[base[b] + r] = list[t];
        __syncthreads();
    }
}
}  // namespace

hipError_t launch_fix_order(const TraceJob *jobs_dev, const FixEntry *list, const uint32_t *count,
                            int64_t cap, int32_t *key, uint32_t *counts, FixEntry *out,
                            hipStream_t s)
{
    int64_t b = (cap + 255) / 256;
    if (b < 1) b = 1;
    if (b > 1024) b = 1024;
    hipLaunchKernelGGL(fill_counts_kernel, dim3(1), dim3(256), 0, s, counts);
    hipLaunchKernelGGL(fix_key_kernel, dim3((unsigned)b), dim3(256), 0, s, jobs_dev, list, count, cap,
                       key, counts);
    hipLaunchKernelGGL(tile_scan_kernel, dim3(1), dim3(64), 0, s, counts);
    hipLaunchKernelGGL(fix_place_kernel, dim3((unsigned)b), dim3(256), 0, s, list, count, cap, key,
                       counts, out);
    return hipGetLastError();
}

hipError_t launch_graze(const TraceJob *jobs_dev, int job, int64_t max_lines, double thr,
                        const double *qmap, double qthr, FixEntry *list, uint32_t *count,
                        uint32_t *count_tw, int64_t cap, int split, int seed_check, hipStream_t s)
{
    int64_t b = (max_lines + 255) / 256;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    hipLaunchKernelGGL(graze_kernel, dim3((unsigned)b), dim3(256), 0, s, jobs_dev, job, thr, qmap,
                       qthr, list, count, count_tw, cap, split, seed_check);
    return hipGetLastError();
}

namespace {
// Copies one job descriptor (a kernel argument) into the device job table, so the
// table lives in the caller's workspace and a captured graph holds no host pointer.
__global__ void store_job_kernel(TraceJob j, TraceJob *dst)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = j;
}
}  // namespace

hipError_t launch_store_job(const TraceJob &j, TraceJob *dst, hipStream_t s)
{
    hipLaunchKernelGGL(store_job_kernel, dim3(1), dim3(64), 0, s, j, dst);
    return hipGetLastError();
}

}  // namespace fq
