/*
 * FP64 CPU oracle: field-line tracing, twist number and squashing factor Q.
 *
 * TEST INFRASTRUCTURE. Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg load this library; the product path never does. It shares no
 * source, header, table or helper with the HIP library.
 *
 * Conventions
 *   - Field: three node planes Bx, By, Bz of n[0] x n[1] x n[2] float64 values,
 *     x fastest: node (i,j,k) at ((k*n[1] + j)*n[0] + i). Node (i,j,k) sits at
 *     origin + (i,j,k) * spacing (uniform Cartesian grid, Section 2.2), or, along
 *     an axis given by its node coordinates, at those (stretched rectilinear grid).
 *   - Lengths are physical (the units of origin/spacing); tolerances are in grid
 *     spacings (the unit the paper uses for tol, Section 2.3): on a stretched grid,
 *     in the widths of the cell the step is taken in.
 *   - Faces of the box: 0 = x-, 1 = x+, 2 = y-, 3 = y+, 4 = z-, 5 = z+.
 */
#ifndef FQ_ORACLE_H
#define FQ_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status bits (per line, OR-ed per map point) */
#define ORC_OK 0
#define ORC_OUTSIDE 1     /* seed outside the box */
#define ORC_NULLB 2       /* |B| vanished on the line */
#define ORC_MAXSTEPS 4    /* step budget exhausted */
#define ORC_NONFINITE 8   /* NaN/Inf met in the field */
#define ORC_ONESIDED 16   /* a one-sided difference was used */
#define ORC_MIXEDFACE 32  /* no neighbour ends on the same faces: Q = NaN */
#define ORC_EDGE 64       /* a line of the stencil ends near a box edge */
#define ORC_ROTATED 128   /* S0 was rotated perpendicular to B */

typedef struct {
    int64_t n[3];
    double origin[3];
    double spacing[3];
    const double *b[3]; /* Bx, By, Bz node planes */
    const double *j[3]; /* curl B node planes (fill with orc_curl) */
    const double *coord[3]; /* stretched axes (Section 2.2): the n[a] node positions,
                               strictly increasing; NULL = uniform (origin + i spacing).
                               On a stretched axis origin and spacing are not used. */
} orc_field;

/* face id of an end on the cylindrical mapping surface (orc_qcyl) */
#define ORC_FACE_CYL 6

/* A cylindrical mapping surface: axis along z through (xc, yc), radius r. */
typedef struct {
    double xc, yc, r;
} orc_cyl;

typedef struct {
    double tol;       /* per-step error bound, grid spacings */
    double h0;        /* first trial step, grid spacings */
    double hmax;      /* largest step, grid spacings */
    int64_t max_steps;/* trial steps per half line */
    double edge_eps;  /* an end closer than this (physical) to a box edge sets ORC_EDGE */
    int want_tw;      /* integrate the twist number */
    int nthreads;     /* OpenMP threads, 0 = runtime default */
} orc_opts;

/* One traced line: the backward (sigma = -1) and forward (sigma = +1) halves. */
typedef struct {
    double *end_b, *end_f;   /* n x 3 end points */
    int8_t *face_b, *face_f; /* n face ids, -1 if none */
    double *bn_b, *bn_f;     /* n: B . e_axis(face) at the ends */
    double *bn0;             /* n: B . normal at the seed (normal given by caller) */
    double *tw, *len;        /* n: whole-line twist number and length */
    uint16_t *status;        /* n */
    int64_t *nsteps;         /* n: accepted steps of both halves (may be NULL) */
} orc_lines;

void orc_default_opts(orc_opts *o);

/* OpenMP threads a parallel region of the oracle uses by default. */
int orc_threads(void);

/* Node-wise curl B by second-order differences (one-sided at the boundary). */
int orc_curl(const orc_field *f, double *jx, double *jy, double *jz);

/* Trilinear interpolant (Eq. interp) of the three planes p at r, in cell c. */
void orc_interp(const orc_field *f, const double *const p[3], const int64_t c[3],
                const double r[3], double out[3]);

/* Trace n seeds (n x 3) both ways; normal (3 doubles, may be NULL = z) sets bn0. */
int orc_trace(const orc_field *f, const double *seeds, int64_t n, const double *normal,
              const orc_opts *o, orc_lines *out);

/* Q, Tw and length on a 2-D seed grid: seed (i,j) = origin + i du u + j dv v. */
int orc_q2d(const orc_field *f, const double origin[3], const double u[3],
            const double v[3], int64_t nu, int64_t nv, double du, double dv,
            const orc_opts *o, double *q, double *tw, double *len, uint16_t *status,
            orc_lines *lines);

/* 3-D maps on voxel centres origin + (i,j,k) spacing; S0 is the z plane through
 * each voxel, rotated perpendicular to B where |Bz/B| < 0.05. */
int orc_q3d(const orc_field *f, const double origin[3], const double spacing[3],
            const int64_t nvox[3], const orc_opts *o, double *q, double *tw,
            double *len, uint16_t *status, orc_lines *lines);

/* The same maps at listed points only (indices into the map, i fastest): each
 * point's line and its stencil neighbours are traced and assembled exactly as in
 * orc_q2d / orc_q3d. Outputs have npts entries. */
int orc_q2d_points(const orc_field *f, const double origin[3], const double u[3],
                   const double v[3], int64_t nu, int64_t nv, double du, double dv,
                   const int64_t *pts, int64_t npts, const orc_opts *o, double *q, double *tw,
                   double *len, uint16_t *status, orc_lines *lines);
int orc_q3d_points(const orc_field *f, const double origin[3], const double spacing[3],
                   const int64_t nvox[3], const int64_t *pts, int64_t npts, const orc_opts *o,
                   double *q, double *tw, double *len, uint16_t *status, orc_lines *lines);

/* Method I on a cylindrical mapping surface (Section 3, the x^2 + y^2 = 1 example):
 * seeds at (xc + r cos theta, yc + r sin theta, z), theta = theta0 + i dtheta
 * (i < ntheta, fastest), z = z0 + j dz. Lines run inside the cylinder only: the
 * half whose direction points out of the cylinder ends at its seed, the other ends
 * where it meets the cylinder again (face ORC_FACE_CYL) or leaves the box. S0, S1
 * and S2 are the cylinder, with coordinates (r theta, z) and normal fields along the
 * outward normal; Q by Eq. D+-2, D+-3 and Q+- on the (theta, z) stencil. The
 * cylinder must lie inside the box in x and y. Outputs as orc_q2d's; bn0 in lines
 * is B . the outward normal at the seed. */
int orc_qcyl(const orc_field *f, const orc_cyl *cyl, double theta0, double dtheta,
             int64_t ntheta, double z0, double dz, int64_t nz, const orc_opts *o, double *q,
             double *tw, double *len, uint16_t *status, orc_lines *lines);

/* Method I with S1, S2 rotated perpendicular to B at the line's ends (Q_perp,
 * Section 2.1) on the 2-D seed grid of orc_q2d, from the 3-D end displacements of
 * the same neighbour stencil projected along B onto those planes, and the length
 * edge map fledge = |grad_S0 length| (neighbour differences of the line lengths).
 * Points whose S0 would be rotated (interior S0, |Bn0/B| < 0.05) get NaN and
 * ORC_ROTATED. */
int orc_q2d_perp(const orc_field *f, const double origin[3], const double u[3],
                 const double v[3], int64_t nu, int64_t nv, double du, double dv,
                 const orc_opts *o, double *qperp, double *fledge, uint16_t *status);

/* Method II (Scott 2017; Section 2.1, Eq. rb2, Eq. q_scott) at n seeds: S0 is
 * perpendicular to B at each seed with orthonormal U, V in it; r, U and V are
 * traced both ways (dU/ds = (U . grad)(B/B)); q gets Q with S1, S2 the faces the
 * line ends on and qperp gets Q_perp with S1, S2 perpendicular to B at the ends.
 * way 1: grad(B/B) interpolated from node values by second-order differences
 * (Eq. grad_B); way 2: central differences of B/B at +-0.001 grid spacings on the
 * current cell's interpolant. Outputs (n entries; any may be NULL) as orc_q2d's;
 * lines gets end_b/end_f/face_b/face_f/status. */
int orc_method2(const orc_field *f, const double *seeds, int64_t n, int way, const orc_opts *o,
                double *q, double *qperp, double *tw, double *len, uint16_t *status,
                orc_lines *lines);

#ifdef __cplusplus
}
#endif
#endif
