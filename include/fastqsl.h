/*
 * fastqsl.h — C-ABI of the MI355X field-line tracer for the squashing factor Q and
 * the twist number Tw (Zhang, Chen, Liu & Wang 2022, "FastQSL").
 *
 * The library traces one magnetic field line per seed through a gridded field,
 * with trilinear interpolation (Section 2.2, Eq. interp) and adaptive RKF45
 * stepping (Section 2.3) both ways to the box faces (Section 2.1), integrates the
 * twist number along it (Section 1, Eq. tw), and forms Method-I Q from the
 * footpoint mapping of neighbouring seeds (Section 2.1, Eq. D+-2, Eq. D+-3;
 * Section 1, Eq. Q+- with |det D| replaced by |Bn1/Bn2|).
 *
 * Conventions shared by every entry point
 *   - Every array pointer is a DEVICE pointer on the current HIP device, allocated
 *     and owned by the caller; the library keeps no reference after the call.
 *     Struct arguments themselves are host memory and are read during the call.
 *   - Fields are three node planes Bx, By, Bz of n[0] x n[1] x n[2] values, x
 *     fastest: node (i,j,k) of a plane is element (k*n[1] + j)*n[0] + i. Node
 *     (i,j,k) sits at origin + (i,j,k) * spacing (a uniform Cartesian grid).
 *   - Step sizes and tolerances are in grid spacings (the paper's unit for tol,
 *     Section 2.3); positions and lengths are in the units of origin/spacing.
 *   - Box faces are numbered 0 = x-, 1 = x+, 2 = y-, 3 = y+, 4 = z-, 5 = z+.
 *   - Calls only enqueue work on `stream` (a hipStream_t; NULL = the null stream)
 *     and return; they never synchronise, never allocate device memory, and issue
 *     no memset node, so a call can be captured into a HIP graph. Scratch memory
 *     comes from the caller's workspace `ws` of `ws_bytes` bytes (256-byte aligned),
 *     sized by the matching *_workspace_size query with the same arguments.
 *   - Return value: FQ_OK or a negative FQ_E* code (fastqsl_strerror gives text).
 *     Argument errors are detected before anything is enqueued. Per-line problems
 *     never fail a call: they set per-line / per-point status bits and NaN outputs.
 */
#ifndef FASTQSL_H
#define FASTQSL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define FQ_OK 0
#define FQ_EINVAL (-1)       /* a null required pointer or an inconsistent argument */
#define FQ_ENOMEM (-2)       /* workspace smaller than the size query returns */
#define FQ_EHIP (-3)         /* a HIP launch failed */
#define FQ_EUNSUPPORTED (-4) /* a valid but unsupported combination */

/* field storage types */
#define FQ_DT_F32 0
#define FQ_DT_F64 1

/* arithmetic forms */
#define FQ_PREC_F32X 0 /* FP32 tracing and interpolation; FP64 Jacobian, Q ratio, Tw sum,
                          normal fields, and FP64 re-tracing of grazing lines */
#define FQ_PREC_F64 1  /* every step in FP64 */

/* integration schemes (Section 2.3) */
#define FQ_SCHEME_RKF45 0  /* adaptive Fehlberg 4(5): error bound tol_perp |Bn0/B|^1.5 (Eq. tol) */
#define FQ_SCHEME_RK4 1    /* classic RK4 with the fixed step max(step_perp |Bn0/B|, step_min) */
#define FQ_SCHEME_RK4_38 2 /* Kutta's 3/8-rule RK4 with that fixed step */

/* how Q is formed (Section 2.1) */
#define FQ_METHOD_I 0  /* neighbour differences of the footpoint mapping through S0 (Eq. D+-2,
                          Eq. D+-3, Eq. Q+-) */
#define FQ_METHOD_II 1 /* tangent vectors U, V traced with the line from S0 perpendicular to B
                          (Eq. rb2), Q and Q_perp by Eq. q_scott; grad(B/B) analytic on the
                          cell's interpolant (the offset differences of Section 4 taken to a
                          vanishing offset) */

/* per-line / per-point status bits */
#define FQ_ST_OK 0
#define FQ_ST_OUTSIDE 1     /* seed outside the box: outputs NaN */
#define FQ_ST_NULLB 2       /* |B| vanished on the line: outputs NaN */
#define FQ_ST_MAXSTEPS 4    /* trial-step budget exhausted: outputs NaN */
#define FQ_ST_NONFINITE 8   /* NaN/Inf in the field on the line: outputs NaN */
#define FQ_ST_ONESIDED 16   /* a one-sided difference entered Q */
#define FQ_ST_MIXEDFACE 32  /* no neighbour ends on the centre line's faces: Q = NaN */
#define FQ_ST_EDGE 64       /* a line of the stencil ends within edge_eps of a box edge */
#define FQ_ST_ROTATED 128   /* S0 rotated perpendicular to B (|Bn0/B| < 0.05, interior S0) */
#define FQ_ST_NOTAPE 256    /* adjoint calls only: the checkpoint pool ran out before this line
                               was traced (set with FQ_ST_MAXSTEPS; the line has no outputs
                               and no derivative; raise fq_params.tape_steps) */

/* A field: three device planes of n[0]*n[1]*n[2] values of type `dtype`, on a
 * uniform grid (node (i,j,k) at origin + (i,j,k) spacing) or a stretched rectilinear
 * one (Section 2.2): an axis a with coord[a] set has its nodes at coord[a][0..n[a]-1]
 * (device, FP64, strictly increasing and finite; read by the call, which copies
 * nothing). On such an axis origin[a] must be the first node and origin[a] +
 * (n[a]-1) spacing[a] the last (spacing[a] is the mean cell width: the box extent
 * stays known to the host). On a stretched grid the per-step error bound is taken in
 * the widths of the cell the step is in, and the first step of Eq. step is scaled by
 * the seed cell's width along B (Section 2.3, the scaling of step and tol on
 * stretched grids). A field whose node coordinates are not strictly increasing and
 * finite, or do not span the box that origin and spacing give (to 1e-12 of its
 * extent), gives its lines FQ_ST_NONFINITE. Method II takes uniform grids only (else
 * FQ_EUNSUPPORTED). */
typedef struct {
    int64_t n[3];         /* nodes along x, y, z; each in [2, 65535] */
    double origin[3];     /* position of node (0,0,0) */
    double spacing[3];    /* node spacing per axis; > 0 */
    int32_t dtype;        /* FQ_DT_F32 or FQ_DT_F64 */
    int32_t reserved;
    const void *b[3];     /* device: Bx, By, Bz planes */
    const double *coord[3]; /* device, optional: node coordinates of a stretched axis (NULL =
                               uniform axis) */
} fq_field;

/* Tracing parameters (Section 2.3 and the S0 rules of Section 4).
 * For a line whose seed has field angle |Bn0/B| to S0, the first step is
 * max(step_perp |Bn0/B|, step_min) (Eq. step) and the per-step error bound is
 * tol_perp |Bn0/B|^1.5 (Eq. tol), with |Bn0/B| taken no smaller than 0.05 for a
 * seed inside the box (S0 is rotated below that) and no smaller than 1e-9 for a
 * seed on a box face, and the bound no smaller than tol_floor. Zero-valued fields
 * take the documented default. */
typedef struct {
    double tol_perp;   /* RKF45 error bound for a line perpendicular to S0 (grid spacings); default 1e-6 */
    double step_perp;  /* first step for a perpendicular line (grid spacings); default 1 */
    double step_min;   /* smallest first step (grid spacings); default 0.05 */
    double tol_floor;  /* smallest error bound used (grid spacings); default 16 ulp(1) of FP32
                          in the F32X form (whose FP64 pass takes the FP64 default, 1e-14,
                          unless a larger floor is given) and 1e-14 in the F64 form */
    double edge_eps;   /* an end this close to a box edge (units of origin/spacing) sets FQ_ST_EDGE; default 1e-5 */
    int64_t max_steps; /* trial steps per half line; default 200000 */
    int32_t precision; /* FQ_PREC_F32X (default) or FQ_PREC_F64 */
    int32_t want_tw;   /* nonzero: integrate Tw (the curl planes are built) */
    int32_t block;     /* threads per block of the tracer: 64, 128, 192 or 256; 0 = 256 */
    int32_t waves_per_cu; /* resident waves per CU the tracer's grid is sized for; 0 = the most that fit */
    double graze;      /* FQ_PREC_F32X only: both halves of a line whose field makes an angle
                          |Bn/B| below this with S0 at its seed, and a half line whose field
                          makes such an angle with the face it ends on (these turn FP32
                          rounding into large footpoint errors), are traced again in FP64,
                          as is any half line the FP32 pass could not finish; default 0.05,
                          negative = no FP64 pass */
    uint64_t *stats;   /* device, optional: 5 counters ADDED to by the tracer — trial steps,
                          accepted steps, cell fetches, half lines traced, half lines traced
                          again in FP64 (NULL = not collected) */
    void *const *events; /* host, optional: 4 hipEvent_t recorded on the call's stream right
                          before and after the tracer launch, and before and after the FP64
                          pass (for timing the tracer alone; NULL = none) */
    double qfix;       /* FQ_PREC_F32X maps only: a line whose map point has Q above this
                          after the FP32 pass is traced again in FP64 too (for a rotated S0,
                          its four extra lines as well), and Q is formed again (the map
                          amplifies a line's FP32 rounding by about sqrt(Q)); default 300,
                          negative = off. Lines of a call with no Q output are not selected
                          this way */
    int64_t tape_steps; /* adjoint calls only: accepted steps per half line, on average over
                          the map, that the checkpoint pool has room for; default 2048. A half
                          line that finds the pool full gets FQ_ST_NOTAPE | FQ_ST_MAXSTEPS */
    int32_t scheme;    /* FQ_SCHEME_RKF45 (default), FQ_SCHEME_RK4 or FQ_SCHEME_RK4_38. Every
                          step stays in one grid cell and ends on the cell face it reaches, in
                          every scheme; a fixed-step scheme takes its step (Eq. step) between
                          faces. The adjoint calls take all three: their reverse pass holds
                          the recorded step lengths fixed, so with a fixed-step scheme the
                          only state-dependent lengths are those of face landings */
    int32_t method;    /* maps: FQ_METHOD_I (default) or FQ_METHOD_II. Method II traces one line
                          per map point (no stencil neighbours, no rotated S0), with Eq. step /
                          Eq. tol at |Bn0/B| = 1 (its S0 is perpendicular to B), RKF45 only, and
                          in the F32X form without the FP64 passes (FP32 tracing; FP64 end
                          fields and Q); the adjoint calls take Method I only */
    int32_t in_flight; /* FQ_PREC_F32X maps: nonzero when the caller keeps other maps in flight
                          on other streams at the same time. The FP64 pass (a tail of few,
                          long lines) then runs at three waves per SIMD, spilling a little, and
                          takes its half lines longest first (waves of short lines end early),
                          so that the other maps' FP32 passes find room beside its waves: more
                          maps per second in flight, a longer FP64 pass for one map alone.
                          Results are the same bit for bit; default 0 */
    int32_t reserved2; /* must be 0 */
} fq_params;

/* A 2-D seed grid on S0: seed (i, j) = origin + i du u + j dv v, i < nu, j < nv,
 * u and v orthonormal. Map points are stored i fastest. */
typedef struct {
    double origin[3];
    double u[3];
    double v[3];
    int64_t nu, nv;
    double du, dv;
} fq_plane;

/* 3-D seeds at voxel centres origin + (i,j,k) spacing (i fastest). S0 of each
 * voxel is the z plane through it; its stencil neighbours are (i+-1, j, k) and
 * (i, j+-1, k). */
typedef struct {
    double origin[3];
    double spacing[3];
    int64_t n[3];
} fq_voxels;

/* A cylindrical mapping surface (Section 3: the x^2 + y^2 = 1 example): axis along z
 * through `centre`, radius `radius`, inside the box in x and y. Map point (i, j),
 * i < ntheta fastest, is the seed (xc + R cos(t), yc + R sin(t), z) with t = theta0 +
 * i dtheta and z = z0 + j dz. Lines run inside the cylinder (and the box): the half
 * whose direction at the seed points out of the cylinder ends at its seed, the other
 * ends where it meets the cylinder again (face FQ_FACE_CYL) or leaves the box. S0, S1
 * and S2 are the cylinder, with coordinates (R theta, z) and normal fields along its
 * outward normal; Q by Method I (Eq. D+-2, D+-3, Q+-) on the (theta, z) stencil. */
typedef struct {
    double centre[2];
    double radius;
    double theta0, dtheta;
    int64_t ntheta;
    double z0, dz;
    int64_t nz;
} fq_cylinder;

#define FQ_FACE_CYL 6 /* face id of an end on a cylindrical mapping surface */

/* Per-line outputs, n entries each (end_b/end_f are n x 3); any pointer may be
 * NULL. The backward half runs against B, the forward half along it. */
typedef struct {
    double *end_b, *end_f;   /* end points of the backward / forward halves */
    int8_t *face_b, *face_f; /* their box faces (-1 when the half failed) */
    double *bn_b, *bn_f;     /* B . e_axis(face) at the ends, FP64 */
    double *bn0;             /* B . normal at the seed, FP64 */
    double *tw;              /* whole-line twist number */
    double *length;          /* whole-line length */
    uint16_t *status;        /* FQ_ST_* bits of the line */
} fq_lines;

/* Per-point map outputs; any pointer may be NULL. */
typedef struct {
    double *q;          /* squashing factor (NaN where undefined) */
    double *tw;         /* twist number of the point's line */
    double *length;     /* length of the point's line */
    uint16_t *status;   /* FQ_ST_* bits of the point */
    fq_lines lines;     /* the point's own line (NULL members skipped) */
    double *qperp;      /* Q_perp, with S1, S2 perpendicular to B at the ends (Section 2.1).
                           Method II: from U, V. Method I (2-D maps; 3-D maps leave it
                           untouched): the end displacements of Q's neighbour stencil,
                           projected along B onto the planes perpendicular to B at the
                           ends; NaN where S0 is rotated */
    double *fledge;     /* 2-D maps (3-D maps leave it untouched): the length edge map,
                           |grad_S0 length| by the neighbour differences of Q's stencil
                           (dimensionless; large where neighbouring lines part, as at
                           QSLs); NaN where no neighbour is usable or S0 is rotated */
} fq_map;

/* ---------------------------------------------------------------------------------
 * fastqsl_trace — trace n seeds (device, n x 3 doubles) both ways to the box
 * (Section 2.1, Eq. rb; Section 2.2; Section 2.3) and integrate Tw along each line
 * (Section 1, Eq. tw). normal (host, 3 doubles; NULL = +z) defines Bn0 and the
 * Eq. step / Eq. tol scaling of each line.
 * ------------------------------------------------------------------------------- */
size_t fastqsl_trace_workspace_size(const fq_field *f, int64_t n, const fq_params *p);
int fastqsl_trace(const fq_field *f, const double *seeds, int64_t n, const double *normal,
                  const fq_params *p, const fq_lines *out, void *ws, size_t ws_bytes,
                  void *stream);

/* ---------------------------------------------------------------------------------
 * fastqsl_q2d — Q, Tw and length maps on 2-D seed grids (Section 2.1 Method I,
 * Eq. D+-2, Eq. D+-3; Section 1, Eq. Q+-, Eq. tw). njobs >= 1 independent
 * (field, plane, map) triples are traced in ONE persistent launch sharing one line
 * queue, so cubes and seed grids of uneven sizes keep the GPU full. fields,
 * planes and maps are host arrays of njobs entries; map pointers are device
 * pointers of nu*nv entries. S0 on a box face is used as is; on an interior plane
 * S0 is rotated perpendicular to B where |Bn0/B| < 0.05 (Section 4); a batch may
 * mix both kinds.
 * ------------------------------------------------------------------------------- */
size_t fastqsl_q2d_workspace_size(const fq_field *fields, const fq_plane *planes, int njobs,
                                  const fq_params *p);
int fastqsl_q2d(const fq_field *fields, const fq_plane *planes, int njobs, const fq_params *p,
                const fq_map *maps, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------------
 * fastqsl_q3d — Q, Tw and length at voxel centres (Section 1, Eq. qline: one line
 * per voxel, its Q assigned to the voxel), with S0 rotated perpendicular to B
 * where |Bz/B| < 0.05 and four extra lines traced there (Section 4).
 * ------------------------------------------------------------------------------- */
size_t fastqsl_q3d_workspace_size(const fq_field *f, const fq_voxels *v, const fq_params *p);
int fastqsl_q3d(const fq_field *f, const fq_voxels *v, const fq_params *p, const fq_map *map,
                void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------------
 * fastqsl_qcyl — Q, Tw and length on a cylindrical mapping surface (Section 3's
 * x^2 + y^2 = 1 example; Section 2.1's choice of S1, S2): the map of fq_cylinder,
 * ntheta x nz points (theta fastest), by Method I. Both forms; RKF45 only (else
 * FQ_EUNSUPPORTED); map->qperp and map->fledge are left untouched. Lines are
 * reported as for fastqsl_q2d, with bn0 = B . the outward normal at the seed and
 * face FQ_FACE_CYL for ends on the cylinder (bn_b/bn_f then along its outward
 * normal). Errors: FQ_EINVAL for a cylinder that is empty, has a radius that is not
 * positive and finite, or leaves the box in x or y.
 * ------------------------------------------------------------------------------- */
size_t fastqsl_qcyl_workspace_size(const fq_field *f, const fq_cylinder *c, const fq_params *p);
int fastqsl_qcyl(const fq_field *f, const fq_cylinder *c, const fq_params *p, const fq_map *map,
                 void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------------
 * fastqsl_backward — reverse-mode derivative of one q2d map with respect to the
 * field's node values. Not an operation of the paper: it differentiates the map of
 * fastqsl_q2d (Section 2.1 tracing and Method-I Q, Eq. D+-2 / D+-3 / Q+-; Tw of
 * Eq. tw) so that a field model can be fitted to target maps.
 *   f, pl, p   the same inputs as the forward call; p->method must be
 *              FQ_METHOD_I (any p->scheme on a plane on a box face; RKF45 on an
 *              interior plane, whose rotated-S0 lines (Section 4) are differentiated
 *              too, their seeds' dependence on B0 included), on a uniform or
 *              stretched grid, else FQ_EUNSUPPORTED. Use the forward call's
 *              parameters: the lines are traced again with them.
 *              p->precision picks the form differentiated: FQ_PREC_F64, or
 *              FQ_PREC_F32X, whose FP32 pass is kept, replayed and reversed in FP32
 *              (the map is the F32X map; half lines that its FP64 pass re-traced take
 *              their derivative from their FP32 trace, and a half line the FP32 pass
 *              could not finish has none and counts as a replay mismatch).
 *   segment    accepted steps between checkpoints, 1..4096.
 *   dq, dtw    dL/dQ and dL/dTw, nu*nv device doubles each (map order), or NULL;
 *   dend_b, dend_f  dL/d(end points), nu*nv x 3 device doubles each, or NULL.
 *              Non-finite entries and points with a failed line are ignored;
 *              points whose Q is NaN contribute no dL/dQ.
 *   gb         three device double planes shaped like the field: dL/dBx, dL/dBy,
 *              dL/dBz are ADDED to them.
 *   ws         caller workspace of fastqsl_backward_workspace_size() bytes (256-byte
 *              aligned). It holds a pool of 2 + ceil(p->tape_steps/segment)
 *              checkpoints of 64 bytes per half line of the plane (shared by all half
 *              lines: room for p->tape_steps accepted steps per half line on
 *              average; an interior plane adds two per potential half line of its
 *              rotated-S0 job), per-half adjoints, node gradients, replay buffers
 *              and the reverse pass's queue order (half lines by accepted steps, most
 *              first).
 * The lines are traced again with the lane state kept every `segment` accepted
 * steps; each segment is then replayed from its checkpoint with the same stepping
 * code and its accepted steps are differentiated last to first (the discrete
 * adjoint with the step lengths held fixed). A half line that finds the pool
 * exhausted is not traced further: it ends with FQ_ST_NOTAPE | FQ_ST_MAXSTEPS, so
 * its point has no outputs and contributes nothing; fastqsl_q2d_record reports
 * those points in the map's status. If p->stats is set, stats[0..3] get the half
 * lines differentiated, the accepted steps reversed, the replays that failed to
 * reproduce the forward pass (expected 0) and the half lines with a nonzero
 * adjoint that were dropped (expected 0).
 * Asynchronous on `stream`; allocates nothing.
 * ------------------------------------------------------------------------------- */
size_t fastqsl_backward_workspace_size(const fq_field *f, const fq_plane *pl,
                                       const fq_params *p, int segment);
int fastqsl_backward(const fq_field *f, const fq_plane *pl, const fq_params *p, int segment,
                     const double *dq, const double *dtw, const double *dend_b,
                     const double *dend_f, double *const gb[3], void *ws, size_t ws_bytes,
                     void *stream);

/* ---------------------------------------------------------------------------------
 * fastqsl_q2d_record, fastqsl_backward_recorded — fastqsl_backward in two calls, for
 * callers that need the map before they know its gradient (a training step: map,
 * loss, then derivative). The lines are traced once.
 *   fastqsl_q2d_record: the checkpointed forward pass of fastqsl_backward, and the
 *     map of fastqsl_q2d (in the form p->precision picks) written to `map` (the same
 *     values fastqsl_q2d writes, bit for bit:
 *     Section 2.1 tracing and Method-I Q, Eq. D+-2 / D+-3 / Q+-; Tw of Eq. tw).
 *   fastqsl_backward_recorded: the reverse pass of fastqsl_backward (same argument
 *     meanings), reading the checkpoints and half-line records the record call left
 *     in `ws`.
 * Both take f, pl, p and segment as fastqsl_backward does and the workspace of
 * fastqsl_backward_workspace_size(); the reverse call must get the same inputs and
 * a workspace that nothing else wrote since the record call, on the same stream (or
 * after it). A record call may be followed by any number of reverse calls. Errors
 * as fastqsl_backward; the map's points follow fastqsl_q2d. Asynchronous on
 * `stream`; allocate nothing.
 * ------------------------------------------------------------------------------- */
int fastqsl_q2d_record(const fq_field *f, const fq_plane *pl, const fq_params *p, int segment,
                       const fq_map *map, void *ws, size_t ws_bytes, void *stream);
int fastqsl_backward_recorded(const fq_field *f, const fq_plane *pl, const fq_params *p,
                              int segment, const double *dq, const double *dtw,
                              const double *dend_b, const double *dend_f, double *const gb[3],
                              void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------------
 * fastqsl_q3d_backward, fastqsl_q3d_record, fastqsl_q3d_backward_recorded — the
 * same three calls for the map of fastqsl_q3d (Section 1, Eq. qline: Q, Tw and
 * length at voxel centres; Section 4: S0 rotated perpendicular to B where
 * |Bz/B| < 0.05, the four extra lines and their seeds' dependence on B0
 * differentiated as on an interior plane).
 *   f, vx, p   the forward call's inputs; p->method FQ_METHOD_I and p->scheme
 *              FQ_SCHEME_RKF45, else FQ_EUNSUPPORTED; either precision form; uniform
 *              or stretched grid.
 *   segment, dq, dtw, dend_b, dend_f, gb  as for fastqsl_backward, with
 *              nx*ny*nz voxels in map order (x fastest, then y, then z).
 *   ws         of fastqsl_q3d_backward_workspace_size() bytes (256-byte aligned):
 *              the checkpoint pool holds 2 + ceil(p->tape_steps/segment)
 *              checkpoints per half line of the voxel centres plus two per potential
 *              half line of the rotated-S0 job, and the rest as for fastqsl_backward.
 * fastqsl_q3d_record writes the map of fastqsl_q3d (bit for bit) with the
 * checkpoints; fastqsl_q3d_backward_recorded reverses them. Workspace rules, stats
 * and errors as for fastqsl_backward and its two-call form. Asynchronous on
 * `stream`; allocate nothing.
 * ------------------------------------------------------------------------------- */
size_t fastqsl_q3d_backward_workspace_size(const fq_field *f, const fq_voxels *vx,
                                           const fq_params *p, int segment);
int fastqsl_q3d_backward(const fq_field *f, const fq_voxels *vx, const fq_params *p, int segment,
                         const double *dq, const double *dtw, const double *dend_b,
                         const double *dend_f, double *const gb[3], void *ws, size_t ws_bytes,
                         void *stream);
int fastqsl_q3d_record(const fq_field *f, const fq_voxels *vx, const fq_params *p, int segment,
                       const fq_map *map, void *ws, size_t ws_bytes, void *stream);
int fastqsl_q3d_backward_recorded(const fq_field *f, const fq_voxels *vx, const fq_params *p,
                                  int segment, const double *dq, const double *dtw,
                                  const double *dend_b, const double *dend_f,
                                  double *const gb[3], void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------------
 * fastqsl_q2d_static — fastqsl_q2d for callers that cannot allocate device memory
 * (code under HIP graph capture that must not allocate, tight serving loops,
 * harnesses that forbid hipMalloc). Same arguments and results as fastqsl_q2d,
 * without the workspace: the scratch is the library's own device array of
 * fastqsl_static_scratch_bytes() (64 MiB), one per GPU, held from the library's
 * load until the process ends. Calls whose fastqsl_q2d_workspace_size exceeds it
 * return FQ_ENOMEM (use fastqsl_q2d with a caller workspace); invalid arguments
 * return FQ_EINVAL. The call allocates nothing and clears the counters it uses
 * itself; calls that overlap on one GPU (two streams or threads) share that
 * GPU's array and race.
 * ------------------------------------------------------------------------------- */
size_t fastqsl_static_scratch_bytes(void);
int fastqsl_q2d_static(const fq_field *fields, const fq_plane *planes, int njobs,
                       const fq_params *p, const fq_map *maps, void *stream);

/* Text of a return code (static storage). */
const char *fastqsl_strerror(int code);

/* Library version string (static storage). */
const char *fastqsl_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FASTQSL_H */
