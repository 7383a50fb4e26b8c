/*
 * FP64 CPU oracle for FastQSL-style field-line tracing (Zhang et al. 2022).
 *
 * TEST INFRASTRUCTURE: loaded only by the tests, the smoke check and the
 * benchmark's CPU-baseline leg. It is never on the product path and shares no
 * code with the HIP library.
 *
 * What it computes
 *   - The magnetic field at any point is the trilinear interpolant of the node
 *     values (Section 2.2, Eq. interp / w0 / w1). Inside one grid cell this is a
 *     polynomial; across cell faces it is only continuous. Grids are uniform or
 *     stretched rectilinear (per axis node coordinates; the cell of a point by
 *     bisection, Section 2.2), and on a stretched axis derivatives at nodes are
 *     those of the quadratic through three nodes.
 *   - A field line solves dr/ds = B/|B| (Section 2.1, Eq. rb). The oracle
 *     approximates the exact solution of that ODE in the interpolated field: it
 *     integrates cell by cell with every step confined to one closed cell (the
 *     cell's own polynomial is used for all stages), and a step that would leave
 *     the cell is cut back so that it ends exactly on the face it crosses first.
 *     Within a cell the right-hand side is smooth, so the integrator keeps its full
 *     order. The integrator is classic RK4 with step doubling and Richardson
 *     extrapolation, the step controlled against a tolerance in grid spacings.
 *   - Lines run both ways from the seed until they leave the box; the end point is
 *     the exact intersection with the box face (the paper's boundary rule,
 *     Section 2.1, read as "land on the face").
 *   - The twist number Tw = integral of (curl B . B)/(4 pi B^2) dl (Section 1,
 *     Eq. tw) is an extra component of the same ODE, curl B being node-wise
 *     second-order differences (the stencil of Eq. grad_B, Section 4) interpolated
 *     like B. The line length is another component.
 *   - On a cylindrical mapping surface (Section 3's x^2 + y^2 = 1 example) lines
 *     run inside the cylinder and end where they meet it again (the crossing found
 *     like a face landing, on the root of phi = r^2 - R^2); Q by Method I on the
 *     surface coordinates (R theta, z).
 *   - Q_perp (S1, S2 perpendicular to B at the ends) by Method I projects the end
 *     displacements of the same stencil along B onto those planes; the length
 *     edge map is |grad_S0 length| on the same stencil.
 *   - Q follows Method I (Section 2.1, Eq. D+-2 and Eq. D+-3): the Jacobians of
 *     both end maps with respect to the seed-plane coordinates come from
 *     differences over neighbouring seeds, D12 = D20 (D10)^-1 with the inverse
 *     written as in Eq. D+-3, and Q = (a^2+b^2+c^2+d^2)/|Bn1/Bn2| (Section 1,
 *     Eq. Q+- with |det D| replaced by the normal-field ratio).
 *
 * How it is pinned (CPU tests, against facts other than itself): exact curl on
 * quadratic fields; trilinear values against an independent interpolator; closed
 * forms of the mapping, Q and Tw in uniform, tilted, sheared, hyperbolic and
 * twisted fields; lines crossing a cell face and back within one step; Q = 2 on
 * arcades over a polarity inversion line of the seed face, down to seeds 1e-8 from
 * it (grazing landings); interior seed planes against the direct S1 -> S2 map;
 * the linear-field closed forms again on stretched grids (cells up to five times
 * their neighbours' width), exact curl and scipy's trilinear interpolation there,
 * seeds on node planes, and explicit uniform nodes against the uniform grid;
 * Method I's Q_perp and the length edge map against the uniform, tilted and
 * sheared closed forms, and Q_perp against Method II's on the charge cube; the
 * cylindrical mapping surface against the paper's B = (x, -y, 0) example (Q = 2,
 * theta2 = pi/2 - theta1, hyperbola arc lengths by scipy) and a tilted uniform
 * field (Q = 2 + 4 bz^2 sin^2 theta1, across the wrap of theta);
 * the rotated S0 of 3-D maps against the closed form of an oblique sheared field,
 * including a voxel with Bz = 0; voxels of two layers of a 3-D map on one line
 * (same Tw and length; Q in the ratio that the interpolant's divergence along
 * the line fixes, computed independently); Q(x1,y1) = Q(x2,y2); flux
 * conservation of the difference Jacobian; B -> -B and mirror symmetries; the
 * paper's quadrupole example (Section 3.2); end points against an independent
 * high-order integrator. Parity unpinned: Q and Tw of the charge and flux-tube
 * benchmark fields themselves, which have no closed form (covered only through
 * the invariances above).
 */
#include "fq_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define FATAL_BITS (ORC_OUTSIDE | ORC_NULLB | ORC_MAXSTEPS | ORC_NONFINITE)

void orc_default_opts(orc_opts *o)
{
    o->tol = 1e-10;
    o->h0 = 0.25;
    o->hmax = 2.0;
    o->max_steps = 1000000;
    o->edge_eps = 1e-5;
    o->want_tw = 1;
    o->nthreads = 0;
}

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int64_t node(const orc_field *f, int64_t i, int64_t j, int64_t k)
{
    return (k * f->n[1] + j) * f->n[0] + i;
}

/* ------------------------------------------------------------------------------
 * curl B at the nodes
 * ---------------------------------------------------------------------------- */

/* Position of node i along axis a (Section 2.2: the nodes x_i, y_j, z_k; on a
 * uniform axis origin + i spacing). */
static double node_x(const orc_field *f, int a, int64_t i)
{
    return f->coord[a] ? f->coord[a][i] : f->origin[a] + (double)i * f->spacing[a];
}

/* Width of cell c along axis a. */
static double cell_w(const orc_field *f, int a, int64_t c)
{
    return f->coord[a] ? f->coord[a][c + 1] - f->coord[a][c] : f->spacing[a];
}

/* Mean cell width along axis a (the spacing of a uniform axis). */
static double mean_w(const orc_field *f, int a)
{
    return f->coord[a] ? (f->coord[a][f->n[a] - 1] - f->coord[a][0]) / (double)(f->n[a] - 1)
                       : f->spacing[a];
}

/* The derivative at x0 of the quadratic through (x0,p0), (x1,p1), (x2,p2): the
 * second-order difference on unequal spacings (Lagrange form). */
static double quad_deriv(double x0, double x1, double x2, double p0, double p1, double p2)
{
    return p0 * (2.0 * x0 - x1 - x2) / ((x0 - x1) * (x0 - x2)) +
           p1 * (x0 - x2) / ((x1 - x0) * (x1 - x2)) + p2 * (x0 - x1) / ((x2 - x0) * (x2 - x1));
}

/* d p / d axis at node (i,j,k): central second-order differences inside, the
 * one-sided second-order formula (-3 f0 + 4 f1 - f2) / 2h on the boundary nodes.
 * On a stretched axis, the same three nodes give the derivative of the quadratic
 * through them (second order on unequal spacings). */
static double deriv(const orc_field *f, const double *p, int axis, int64_t i, int64_t j,
                    int64_t k)
{
    int64_t idx[3] = {i, j, k};
    int64_t n = f->n[axis];
    double h = f->spacing[axis];
    int64_t m = idx[axis];
    int64_t a[3], b[3], c[3];
    memcpy(a, idx, sizeof a);
    memcpy(b, idx, sizeof b);
    memcpy(c, idx, sizeof c);
    if (f->coord[axis]) {
        const double *x = f->coord[axis];
        if (n < 3) {
            a[axis] = 0;
            b[axis] = 1;
            return (p[node(f, b[0], b[1], b[2])] - p[node(f, a[0], a[1], a[2])]) / (x[1] - x[0]);
        }
        /* the three nodes: this one and its two neighbours, or the two inward ones
         * on a boundary node */
        int64_t m1 = m == 0 ? 1 : (m == n - 1 ? n - 2 : m - 1);
        int64_t m2 = m == 0 ? 2 : (m == n - 1 ? n - 3 : m + 1);
        b[axis] = m1;
        c[axis] = m2;
        return quad_deriv(x[m], x[m1], x[m2], p[node(f, a[0], a[1], a[2])],
                          p[node(f, b[0], b[1], b[2])], p[node(f, c[0], c[1], c[2])]);
    }
    if (n < 3) { /* two nodes only: the single first-order difference */
        a[axis] = 0;
        b[axis] = 1;
        return (p[node(f, b[0], b[1], b[2])] - p[node(f, a[0], a[1], a[2])]) / h;
    }
    if (m == 0) {
        b[axis] = 1;
        c[axis] = 2;
        return (-3.0 * p[node(f, a[0], a[1], a[2])] + 4.0 * p[node(f, b[0], b[1], b[2])] -
                p[node(f, c[0], c[1], c[2])]) / (2.0 * h);
    }
    if (m == n - 1) {
        b[axis] = n - 2;
        c[axis] = n - 3;
        return (3.0 * p[node(f, a[0], a[1], a[2])] - 4.0 * p[node(f, b[0], b[1], b[2])] +
                p[node(f, c[0], c[1], c[2])]) / (2.0 * h);
    }
    a[axis] = m - 1;
    b[axis] = m + 1;
    return (p[node(f, b[0], b[1], b[2])] - p[node(f, a[0], a[1], a[2])]) / (2.0 * h);
}

int orc_curl(const orc_field *f, double *jx, double *jy, double *jz)
{
    if (f->n[0] < 2 || f->n[1] < 2 || f->n[2] < 2) return -1;
    const double *bx = f->b[0], *by = f->b[1], *bz = f->b[2];
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t k = 0; k < f->n[2]; k++)
        for (int64_t j = 0; j < f->n[1]; j++)
            for (int64_t i = 0; i < f->n[0]; i++) {
                int64_t q = node(f, i, j, k);
                jx[q] = deriv(f, bz, 1, i, j, k) - deriv(f, by, 2, i, j, k);
                jy[q] = deriv(f, bx, 2, i, j, k) - deriv(f, bz, 0, i, j, k);
                jz[q] = deriv(f, by, 0, i, j, k) - deriv(f, bx, 1, i, j, k);
            }
    return 0;
}

/* ------------------------------------------------------------------------------
 * trilinear interpolation (Eq. interp, w0, w1) in a given cell
 * ---------------------------------------------------------------------------- */

void orc_interp(const orc_field *f, const double *const p[3], const int64_t c[3],
                const double r[3], double out[3])
{
    double w[3][2];
    for (int a = 0; a < 3; a++) {
        double lo = node_x(f, a, c[a]);
        double hi = node_x(f, a, c[a] + 1);
        w[a][0] = (hi - r[a]) / (hi - lo); /* omega_{.,0} */
        w[a][1] = 1.0 - w[a][0];           /* omega_{.,1} */
    }
    for (int comp = 0; comp < 3; comp++) {
        double s = 0.0;
        for (int m = 0; m < 2; m++)
            for (int n = 0; n < 2; n++)
                for (int q = 0; q < 2; q++)
                    s += w[0][m] * w[1][n] * w[2][q] *
                         p[comp][node(f, c[0] + m, c[1] + n, c[2] + q)];
        out[comp] = s;
    }
}

/* The grid cell holding r: floor((r - origin)/spacing), clamped to [0, n-2] so
 * that a point on an upper box face belongs to the last cell; on a stretched axis
 * the last node at or below r, by bisection (Section 2.2). */
static void locate(const orc_field *f, const double r[3], int64_t c[3])
{
    for (int a = 0; a < 3; a++) {
        if (f->coord[a]) {
            int64_t lo = 0, hi = f->n[a] - 1; /* x[lo] <= r < x[hi] kept while possible */
            while (hi - lo > 1) {
                int64_t mid = lo + (hi - lo) / 2;
                if (f->coord[a][mid] <= r[a]) lo = mid;
                else hi = mid;
            }
            if (lo > f->n[a] - 2) lo = f->n[a] - 2;
            c[a] = lo;
            continue;
        }
        double t = floor((r[a] - f->origin[a]) / f->spacing[a]);
        int64_t i = (int64_t)t;
        if (i < 0) i = 0;
        if (i > f->n[a] - 2) i = f->n[a] - 2;
        c[a] = i;
    }
}

static double face_lo(const orc_field *f, const int64_t c[3], int a) { return node_x(f, a, c[a]); }

static double face_hi(const orc_field *f, const int64_t c[3], int a)
{
    return node_x(f, a, c[a] + 1);
}

static double box_lo(const orc_field *f, int a) { return node_x(f, a, 0); }

static double box_hi(const orc_field *f, int a) { return node_x(f, a, f->n[a] - 1); }

/* The smallest cell width of the grid (the reference length of steps). */
static double min_width(const orc_field *f)
{
    double d = INFINITY;
    for (int a = 0; a < 3; a++) {
        if (!f->coord[a]) {
            if (f->spacing[a] < d) d = f->spacing[a];
            continue;
        }
        for (int64_t c = 0; c + 1 < f->n[a]; c++)
            if (cell_w(f, a, c) < d) d = cell_w(f, a, c);
    }
    return d;
}

static int in_box(const orc_field *f, const double r[3])
{
    for (int a = 0; a < 3; a++)
        if (!(r[a] >= box_lo(f, a) && r[a] <= box_hi(f, a))) return 0;
    return 1;
}

/* ------------------------------------------------------------------------------
 * the line ODE (Eq. rb) with the twist integrand (Eq. tw) and length
 * y = (x, y, z, Tw, l);  dy/ds = (sigma B/|B|, (curl B . B)/(4 pi |B|^2), 1)
 * ---------------------------------------------------------------------------- */

/* State of a line: y = (x, y, z, Tw, l) for Method I, followed by the two tangent
 * vectors U, V of Method II (Section 2.1, Eq. rb2): NY components in all. */
#define NY 11

typedef struct {
    const orc_field *f;
    int64_t c[3];
    int sigma;
    int want_tw;
    double bnull2; /* |B|^2 below this counts as a null */
    int nq;        /* components integrated: 5 (Method I) or NY (Method II) */
    int way;       /* Method II: 1 = node array of grad(B/B) (gb), 2 = offset differences */
    const double *const *gb; /* way 1: the 9 planes d(B_i/B)/dx_j, plane 3 i + j */
} line_ctx;

/* The unit vector B/|B| of the current cell's interpolant at r. */
static int unit_b(const line_ctx *L, const double r[3], double b[3])
{
    double B[3];
    orc_interp(L->f, L->f->b, L->c, r, B);
    double bm = sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
    if (!isfinite(bm)) return ORC_NONFINITE;
    if (bm * bm <= L->bnull2) return ORC_NULLB;
    for (int a = 0; a < 3; a++) b[a] = B[a] / bm;
    return 0;
}

/* The Jacobian g[i][j] = d(B_i/B)/dx_j at r (Section 4, Eq. grad_B and the text
 * around it): way 1 interpolates the node array (Eq. interp in the current cell);
 * way 2 takes central differences of B/B at r +- 0.001 grid spacings along each
 * axis, on the current cell's interpolant. */
static int grad_b(const line_ctx *L, const double r[3], double g[3][3])
{
    if (L->way == 1) {
        for (int i = 0; i < 3; i++) {
            const double *const p[3] = {L->gb[3 * i], L->gb[3 * i + 1], L->gb[3 * i + 2]};
            orc_interp(L->f, p, L->c, r, g[i]);
        }
        return 0;
    }
    for (int j = 0; j < 3; j++) {
        double h = 1e-3 * cell_w(L->f, j, L->c[j]);
        double rp[3] = {r[0], r[1], r[2]}, rm[3] = {r[0], r[1], r[2]}, bp[3], bm[3];
        rp[j] += h;
        rm[j] -= h;
        int st;
        if ((st = unit_b(L, rp, bp)) || (st = unit_b(L, rm, bm))) return st;
        for (int i = 0; i < 3; i++) g[i][j] = (bp[i] - bm[i]) / (2.0 * h);
    }
    return 0;
}

static int rhs(const line_ctx *L, const double y[NY], double dy[NY])
{
    double B[3];
    orc_interp(L->f, L->f->b, L->c, y, B);
    double b2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
    if (!isfinite(b2)) return ORC_NONFINITE;
    if (b2 <= L->bnull2) return ORC_NULLB;
    double bm = sqrt(b2);
    for (int a = 0; a < 3; a++) dy[a] = (double)L->sigma * B[a] / bm;
    dy[3] = 0.0;
    if (L->want_tw) {
        double J[3];
        orc_interp(L->f, L->f->j, L->c, y, J);
        double jb = J[0] * B[0] + J[1] * B[1] + J[2] * B[2];
        if (!isfinite(jb)) return ORC_NONFINITE;
        dy[3] = jb / (4.0 * M_PI * b2);
    }
    dy[4] = 1.0;
    if (L->nq > 5) {
        /* Eq. rb2: dU/ds = (U . grad)(B/B), the same for V, along the direction the
         * half line runs (sigma) */
        double g[3][3];
        int st = grad_b(L, y, g);
        if (st) return st;
        for (int i = 0; i < 3; i++) {
            double du = 0.0, dv = 0.0;
            for (int j = 0; j < 3; j++) {
                du += g[i][j] * y[5 + j];
                dv += g[i][j] * y[8 + j];
            }
            dy[5 + i] = (double)L->sigma * du;
            dy[8 + i] = (double)L->sigma * dv;
        }
        for (int q = 5; q < NY; q++)
            if (!isfinite(dy[q])) return ORC_NONFINITE;
    }
    return 0;
}

/* one classic RK4 step of length t */
static int rk4(const line_ctx *L, const double y[NY], double t, double out[NY])
{
    double k1[NY], k2[NY], k3[NY], k4[NY], z[NY];
    int st, n = L->nq;
    if ((st = rhs(L, y, k1))) return st;
    for (int q = 0; q < n; q++) z[q] = y[q] + 0.5 * t * k1[q];
    if ((st = rhs(L, z, k2))) return st;
    for (int q = 0; q < n; q++) z[q] = y[q] + 0.5 * t * k2[q];
    if ((st = rhs(L, z, k3))) return st;
    for (int q = 0; q < n; q++) z[q] = y[q] + t * k3[q];
    if ((st = rhs(L, z, k4))) return st;
    for (int q = 0; q < n; q++)
        out[q] = y[q] + t / 6.0 * (k1[q] + 2.0 * k2[q] + 2.0 * k3[q] + k4[q]);
    for (int q = n; q < NY; q++) out[q] = y[q];
    return 0;
}

/* Step doubling: one step of t against two of t/2. The difference estimates the
 * error (divided by 2^4 - 1); Richardson extrapolation gives the returned state.
 * err is the position part in grid spacings; for Method II the tangent vectors'
 * parts, relative to their size (at least 1), join it. */
static int rk4_doubled(const line_ctx *L, const double y[NY], double t, double out[NY],
                       double *err)
{
    double one[NY], half[NY], two[NY];
    int st;
    if ((st = rk4(L, y, t, one))) return st;
    if ((st = rk4(L, y, 0.5 * t, half))) return st;
    if ((st = rk4(L, half, 0.5 * t, two))) return st;
    double e2 = 0.0;
    for (int q = 0; q < NY; q++) {
        double d = (two[q] - one[q]) / 15.0;
        out[q] = two[q] + d;
        if (q < 3) {
            double g = d / cell_w(L->f, q, L->c[q]);
            e2 += g * g;
        }
    }
    if (L->nq > 5)
        for (int v = 5; v < NY; v += 3) {
            double m = sqrt(y[v] * y[v] + y[v + 1] * y[v + 1] + y[v + 2] * y[v + 2]);
            if (m < 1.0) m = 1.0;
            for (int q = v; q < v + 3; q++) {
                double d = (two[q] - one[q]) / 15.0 / m;
                e2 += d * d;
            }
        }
    *err = sqrt(e2);
    return 0;
}

/* Length t in (0, t_hi] at which the step from y ends on the plane
 * coordinate[a] = plane; g(0) and g(t_hi) must bracket the root. Illinois-modified
 * regula falsi on g(t) = Phi(y, t)[a] - plane.
 *
 * The iteration stops on the width of the bracket in arc length, not on the size
 * of g: the line moves at unit speed, so a bracket of width w bounds the error of
 * the landed point by w whatever the angle between the line and the plane. (A stop
 * on |g| below a fixed height lets a line that grazes the plane at angle alpha land
 * up to height/alpha away from the crossing; near a polarity inversion line on a
 * box face that error reaches the seed's own distance from the inversion line.) */
static int land(const line_ctx *L, const double y[NY], int a, double plane, double t_hi,
                double g_hi, double out[NY], double *t_out)
{
    double ta = 0.0, ga = y[a] - plane;
    double tb = t_hi, gb = g_hi;
    double err, t = t_hi;
    int side = 0, st;
    double cur[NY];
    memcpy(cur, out, sizeof cur);
    for (int it = 0; it < 400; it++) {
        t = (ta * gb - tb * ga) / (gb - ga);
        if (!(t > ta && t < tb)) t = 0.5 * (ta + tb);
        if ((st = rk4_doubled(L, y, t, cur, &err))) return st;
        double gt = cur[a] - plane;
        if (gt == 0.0 || (tb - ta) <= 1e-15 * t_hi) break;
        if ((gt > 0) == (gb > 0)) {
            tb = t;
            gb = gt;
            if (side == 1) ga *= 0.5;
            side = 1;
        } else {
            ta = t;
            ga = gt;
            if (side == -1) gb *= 0.5;
            side = -1;
        }
    }
    memcpy(out, cur, sizeof cur);
    *t_out = t;
    return 0;
}

/* The cylindrical mapping surface (axis along z): phi < 0 inside, phi = 0 on it. */
static double cyl_phi(const orc_cyl *c, const double y[3])
{
    double dx = y[0] - c->xc, dy = y[1] - c->yc;
    return dx * dx + dy * dy - c->r * c->r;
}

/* Outward unit normal of the cylinder through the point y (radial direction). */
static void cyl_normal(const orc_cyl *c, const double y[3], double n[3])
{
    double dx = y[0] - c->xc, dy = y[1] - c->yc, m = sqrt(dx * dx + dy * dy);
    n[0] = dx / m;
    n[1] = dy / m;
    n[2] = 0.0;
}

/* Length t in (0, t_hi] at which the step from y (inside, phi < 0) reaches the
 * cylinder, phi(Phi(y, t_hi)) = g_hi >= 0: the same Illinois iteration and stop
 * on the bracket's width in arc length as land(). */
static int land_cyl(const line_ctx *L, const orc_cyl *c, const double y[NY], double t_hi,
                    double g_hi, double out[NY], double *t_out)
{
    double ta = 0.0, ga = cyl_phi(c, y);
    double tb = t_hi, gb = g_hi;
    double err, t = t_hi;
    int side = 0, st;
    double cur[NY];
    memcpy(cur, out, sizeof cur);
    if (!(ga < 0.0)) {
        /* a step from the cylinder itself (a seed, phi = 0 to rounding) that ends
         * outside it: the line went inside first (its direction points inward), so
         * the crossing sought is the far root; bracket it with an inside point of
         * the step, halving back towards its start */
        double tt = t_hi;
        for (int k = 0; k < 60 && !(ga < 0.0); k++) {
            tt *= 0.5;
            if ((st = rk4_doubled(L, y, tt, cur, &err))) return st;
            if (cyl_phi(c, cur) < 0.0) ta = tt, ga = cyl_phi(c, cur);
        }
        if (!(ga < 0.0)) {
            memcpy(out, y, sizeof cur);  /* never inside: the line ends at its start */
            *t_out = 0.0;
            return 0;
        }
    }
    for (int it = 0; it < 400; it++) {
        t = (ta * gb - tb * ga) / (gb - ga);
        if (!(t > ta && t < tb)) t = 0.5 * (ta + tb);
        if ((st = rk4_doubled(L, y, t, cur, &err))) return st;
        double gt = cyl_phi(c, cur);
        if (gt == 0.0 || (tb - ta) <= 1e-15 * t_hi) break;
        if ((gt > 0) == (gb > 0)) {
            tb = t;
            gb = gt;
            if (side == 1) ga *= 0.5;
            side = 1;
        } else {
            ta = t;
            ga = gt;
            if (side == -1) gb *= 0.5;
            side = -1;
        }
    }
    memcpy(out, cur, sizeof cur);
    *t_out = t;
    return 0;
}

/* inside the closed cell along every axis except `skip` (-1: none) */
static int inside_cell(const line_ctx *L, const double r[3], int skip)
{
    for (int a = 0; a < 3; a++)
        if (a != skip && (r[a] > face_hi(L->f, L->c, a) || r[a] < face_lo(L->f, L->c, a)))
            return 0;
    return 1;
}

/* First parameter value in (0, t) at which the step y -> y1 (slopes dy0 at the
 * start) leaves the closed cell along an axis other than `skip`, judged at the RK4
 * half step and at 15 points of the cubic Hermite interpolant; 0 if none. */
static double excursion(const line_ctx *L, const double y[NY], const double dy0[NY],
                        const double y1[NY], double t, int skip)
{
    double mid[NY], dy1[NY];
    if (rk4(L, y, 0.5 * t, mid) == 0 && !inside_cell(L, mid, skip)) return 0.5 * t;
    if (rhs(L, y1, dy1)) return 0.0;
    for (int k = 1; k < 16; k++) {
        double th = k / 16.0, th2 = th * th, th3 = th2 * th;
        double h00 = 2 * th3 - 3 * th2 + 1, h10 = th3 - 2 * th2 + th;
        double h01 = -2 * th3 + 3 * th2, h11 = th3 - th2;
        double r[3];
        for (int a = 0; a < 3; a++)
            r[a] = h00 * y[a] + h10 * t * dy0[a] + h01 * y1[a] + h11 * t * dy1[a];
        if (!inside_cell(L, r, skip)) return th * t;
    }
    return 0.0;
}

typedef struct {
    double end[3];
    int face;
    double bn;
    double tw, len;
    int status;
    int64_t nsteps;
    double U[3], V[3]; /* Method II: the tangent vectors at the end */
} half_line;

/* Method II inputs of a half line: how grad(B/B) is taken and the tangent vectors
 * at the seed. */
typedef struct {
    int way;
    const double *const *gb;
    double U0[3], V0[3];
} m2_ctx;

/* Trace one half line (direction sigma) from seed until it leaves the box; with m2,
 * the tangent vectors of Method II ride along (Eq. rb2). */
/* With cyl, the line runs inside the cylinder (and the box) only: a half whose
 * direction at the seed (on the cylinder) points out of it ends at its seed, and a
 * half that reaches the cylinder again ends there (face ORC_FACE_CYL, bn = B . the
 * outward normal). */
static void trace_half_gen(const orc_field *f, const double seed[3], int sigma,
                           const orc_opts *o, double bnull2, const m2_ctx *m2,
                           const orc_cyl *cyl, half_line *res)
{
    line_ctx L;
    L.f = f;
    L.sigma = sigma;
    L.want_tw = o->want_tw;
    L.bnull2 = bnull2;
    L.nq = m2 ? NY : 5;
    L.way = m2 ? m2->way : 0;
    L.gb = m2 ? m2->gb : NULL;
    double dmin = min_width(f);

    double y[NY] = {seed[0], seed[1], seed[2], 0.0, 0.0};
    for (int a = 0; a < 3; a++) {
        y[5 + a] = m2 ? m2->U0[a] : 0.0;
        y[8 + a] = m2 ? m2->V0[a] : 0.0;
        res->U[a] = res->V[a] = NAN;
    }
    res->face = -1;
    res->status = 0;
    res->nsteps = 0;
    res->tw = res->len = NAN;
    res->bn = NAN;
    for (int a = 0; a < 3; a++) res->end[a] = NAN;
    if (!in_box(f, seed)) {
        res->status = ORC_OUTSIDE;
        return;
    }
    locate(f, seed, L.c);
    /* the end of the half on the cylinder at y (its cell L.c) */
#define CYL_END(yy)                                                                        \
    do {                                                                                   \
        double B_[3], n_[3];                                                               \
        orc_interp(f, f->b, L.c, (yy), B_);                                                \
        cyl_normal(cyl, (yy), n_);                                                         \
        memcpy(res->end, (yy), 3 * sizeof(double));                                        \
        res->face = ORC_FACE_CYL;                                                          \
        res->bn = B_[0] * n_[0] + B_[1] * n_[1] + B_[2] * n_[2];                           \
        res->tw = (yy)[3];                                                                 \
        res->len = (yy)[4];                                                                \
        for (int a_ = 0; a_ < 3; a_++) {                                                   \
            res->U[a_] = (yy)[5 + a_];                                                     \
            res->V[a_] = (yy)[8 + a_];                                                     \
        }                                                                                  \
    } while (0)
    if (cyl) {
        double B[3], n[3];
        orc_interp(f, f->b, L.c, seed, B);
        cyl_normal(cyl, seed, n);
        if (sigma * (B[0] * n[0] + B[1] * n[1] + B[2] * n[2]) >= 0.0) {
            CYL_END(y);
            return;
        }
    }
    double h = o->h0 * dmin;
    const double hmax = o->hmax * dmin;
    int64_t trials = 0;
    for (;;) {
        if (++trials > o->max_steps) {
            res->status = ORC_MAXSTEPS;
            return;
        }
        /* a point on a face of its cell, heading out through that face, moves to
         * the neighbouring cell; if there is none the line has left the box */
        double dy[NY];
        int st = rhs(&L, y, dy);
        if (st) {
            res->status = st;
            return;
        }
        int exit_face = -1;
        for (int a = 0; a < 3 && exit_face < 0; a++) {
            if (y[a] == face_hi(f, L.c, a) && dy[a] > 0.0) {
                if (L.c[a] == f->n[a] - 2) exit_face = 2 * a + 1;
                else L.c[a]++;
            } else if (y[a] == face_lo(f, L.c, a) && dy[a] < 0.0) {
                if (L.c[a] == 0) exit_face = 2 * a;
                else L.c[a]--;
            }
        }
        if (exit_face >= 0) {
            double B[3];
            orc_interp(f, f->b, L.c, y, B);
            memcpy(res->end, y, 3 * sizeof(double));
            res->face = exit_face;
            res->bn = B[exit_face / 2];
            res->tw = y[3];
            res->len = y[4];
            for (int a = 0; a < 3; a++) {
                res->U[a] = y[5 + a];
                res->V[a] = y[8 + a];
            }
            return;
        }

        /* trial step within the current cell's polynomial */
        double y1[NY], err;
        if ((st = rk4_doubled(&L, y, h, y1, &err))) {
            res->status = st;
            return;
        }
        if (err > o->tol) {
            double s = 0.9 * pow(o->tol / err, 0.2);
            h *= (s < 0.1 ? 0.1 : s);
            continue;
        }
        /* accepted: does it stay in the closed cell? */
        int out_axis[3] = {0, 0, 0}, any = 0;
        for (int a = 0; a < 3; a++) {
            if (y1[a] > face_hi(f, L.c, a)) out_axis[a] = 1, any = 1;
            else if (y1[a] < face_lo(f, L.c, a)) out_axis[a] = -1, any = 1;
        }
        if (!any) {
            /* the end is inside, but the line may have left the cell and come back
             * within the step: look at the half step and at points of the cubic
             * Hermite interpolant of the step; if one is outside, retry with the step
             * cut at the first such point */
            double t_out = excursion(&L, y, dy, y1, h, -1);
            if (t_out > 0.0) {
                h = t_out;
                continue;
            }
            if (cyl && cyl_phi(cyl, y1) > 0.0) {
                /* the step leaves the cylinder: end on it */
                double yc_[NY], tc;
                memcpy(yc_, y1, sizeof yc_);
                if ((st = land_cyl(&L, cyl, y, h, cyl_phi(cyl, y1), yc_, &tc))) {
                    res->status = st;
                    return;
                }
                CYL_END(yc_);
                return;
            }
            memcpy(y, y1, sizeof y);
            res->nsteps++;
            double s = (err > 0.0) ? 0.9 * pow(o->tol / err, 0.2) : 4.0;
            h *= (s > 4.0 ? 4.0 : s);
            if (h > hmax) h = hmax;
            continue;
        }
        /* the step leaves the cell: shorten it to end on the first face crossed
         * (ties go to the lower axis) */
        double t_best = h, y_best[NY];
        int a_best = -1;
        for (int a = 0; a < 3; a++) {
            if (!out_axis[a]) continue;
            double plane = out_axis[a] > 0 ? face_hi(f, L.c, a) : face_lo(f, L.c, a);
            double ya[NY], ta;
            memcpy(ya, y1, sizeof ya);
            if ((st = land(&L, y, a, plane, h, y1[a] - plane, ya, &ta))) {
                res->status = st;
                return;
            }
            if (a_best < 0 || ta < t_best) {
                t_best = ta;
                a_best = a;
                memcpy(y_best, ya, sizeof ya);
                y_best[a] = plane;
            }
        }
        /* A face crossed and crossed back within the trial step leaves its end inside
         * along that axis, so the landing above may have found a later face: the
         * landed point then lies beyond that face by more than the root tolerance.
         * The line left through it first; land on it instead (each pass shortens the
         * step, so this ends). */
        for (int pass = 0; pass < 8; pass++) {
            int a_out = -1;
            double plane = 0.0;
            for (int a = 0; a < 3 && a_out < 0; a++) {
                if (a == a_best) continue;
                double slack = 1e-12 * cell_w(f, a, L.c[a]);
                if (y_best[a] > face_hi(f, L.c, a) + slack) a_out = a, plane = face_hi(f, L.c, a);
                else if (y_best[a] < face_lo(f, L.c, a) - slack) a_out = a, plane = face_lo(f, L.c, a);
            }
            if (a_out < 0) break;
            double ya[NY], ta;
            memcpy(ya, y_best, sizeof ya);
            if ((st = land(&L, y, a_out, plane, t_best, y_best[a_out] - plane, ya, &ta))) {
                res->status = st;
                return;
            }
            t_best = ta;
            a_best = a_out;
            memcpy(y_best, ya, sizeof ya);
            y_best[a_out] = plane;
        }
        /* the shortened step must not leave the cell along another axis on the way
         * (a brief excursion over a neighbouring face): cut it there instead */
        {
            double t_out = excursion(&L, y, dy, y_best, t_best, a_best);
            if (t_out > 0.0) {
                h = t_out;
                continue;
            }
        }
        /* keep the landed point in the closed cell (root tolerance only) */
        for (int a = 0; a < 3; a++) {
            if (a == a_best) continue;
            double lo = face_lo(f, L.c, a), hi = face_hi(f, L.c, a);
            if (y_best[a] < lo) y_best[a] = lo;
            if (y_best[a] > hi) y_best[a] = hi;
        }
        if (cyl && cyl_phi(cyl, y_best) > 0.0) {
            /* the line meets the cylinder before this cell face: end on it */
            double yc_[NY], tc;
            memcpy(yc_, y_best, sizeof yc_);
            if ((st = land_cyl(&L, cyl, y, t_best, cyl_phi(cyl, y_best), yc_, &tc))) {
                res->status = st;
                return;
            }
            CYL_END(yc_);
            return;
        }
        memcpy(y, y_best, sizeof y);
        res->nsteps++;
    }
#undef CYL_END
}


/* in-face coordinates of an end point on face `face`: the two other axes, in
 * increasing axis order */
static void inface(int face, const double e[3], double uv[2])
{
    int a = face / 2, m = 0;
    for (int b = 0; b < 3; b++)
        if (b != a) uv[m++] = e[b];
}

/* In-surface coordinates of an end: in-face ones on a box face, (r theta, z) on the
 * cylinder (arc length around the axis from the +x direction, and height). */
static void surf_uv(const orc_cyl *cyl, int face, const double e[3], double uv[2])
{
    if (face != ORC_FACE_CYL) {
        inface(face, e, uv);
        return;
    }
    uv[0] = cyl->r * atan2(e[1] - cyl->yc, e[0] - cyl->xc);
    uv[1] = e[2];
}

/* The arc length u shifted by whole turns to lie within half a turn of ref. */
static double unwrap(const orc_cyl *cyl, double u, double ref)
{
    double turn = 2.0 * M_PI * cyl->r;
    while (u - ref > 0.5 * turn) u -= turn;
    while (ref - u > 0.5 * turn) u += turn;
    return u;
}

static int near_edge(const orc_field *f, int face, const double e[3], double eps)
{
    if (face < 0) return 0;
    /* the cylinder (inside the box in x and y) meets only the z faces */
    if (face == ORC_FACE_CYL) return e[2] - box_lo(f, 2) < eps || box_hi(f, 2) - e[2] < eps;
    int a = face / 2;
    for (int b = 0; b < 3; b++) {
        if (b == a) continue;
        if (e[b] - box_lo(f, b) < eps || box_hi(f, b) - e[b] < eps) return 1;
    }
    return 0;
}

static double field_scale2(const orc_field *f)
{
    int64_t nn = f->n[0] * f->n[1] * f->n[2];
    double m = 0.0;
    for (int64_t q = 0; q < nn; q++) {
        double b2 = f->b[0][q] * f->b[0][q] + f->b[1][q] * f->b[1][q] +
                    f->b[2][q] * f->b[2][q];
        if (b2 > m) m = b2;
    }
    return m;
}

/* both halves of one line + B . normal at the seed */
typedef struct {
    double end_b[3], end_f[3];
    int face_b, face_f;
    double bn_b, bn_f, bn0;
    double tw, len;
    double len_b, len_f;
    int status;
    int64_t nsteps;
} full_line;

/* The two ends in the order used for S1 and S2. Normally S1 is the backward end
 * and S2 the forward end. For a seed on a box face one half has zero length (the
 * seed is its own end); that end is S1, whatever the polarity, so that
 * neighbouring seeds on both sides of a polarity inversion line difference the
 * same map (the seed -> far footpoint map). Q is symmetric in S1 <-> S2. */
typedef struct {
    const double *e1, *e2;
    int f1, f2;
    double bn1, bn2;
} ends12;

static ends12 order_ends(const full_line *l)
{
    ends12 r;
    int swap = (l->len_f == 0.0 && l->len_b != 0.0);
    r.e1 = swap ? l->end_f : l->end_b;
    r.e2 = swap ? l->end_b : l->end_f;
    r.f1 = swap ? l->face_f : l->face_b;
    r.f2 = swap ? l->face_b : l->face_f;
    r.bn1 = swap ? l->bn_f : l->bn_b;
    r.bn2 = swap ? l->bn_b : l->bn_f;
    return r;
}

/* Both halves from seed; with cyl, inside that cylinder (the S0 normal at the seed
 * is then the cylinder's). */
static void trace_full_gen(const orc_field *f, const double seed[3], const double nrm[3],
                           const orc_cyl *cyl, const orc_opts *o, double bnull2, full_line *r)
{
    half_line hb, hf;
    trace_half_gen(f, seed, -1, o, bnull2, NULL, cyl, &hb);
    trace_half_gen(f, seed, +1, o, bnull2, NULL, cyl, &hf);
    memcpy(r->end_b, hb.end, sizeof r->end_b);
    memcpy(r->end_f, hf.end, sizeof r->end_f);
    r->face_b = hb.face;
    r->face_f = hf.face;
    r->bn_b = hb.bn;
    r->bn_f = hf.bn;
    r->status = hb.status | hf.status;
    r->nsteps = hb.nsteps + hf.nsteps;
    r->tw = hb.tw + hf.tw;
    r->len = hb.len + hf.len;
    r->len_b = hb.len;
    r->len_f = hf.len;
    r->bn0 = NAN;
    if (!(r->status & ORC_OUTSIDE)) {
        int64_t c[3];
        double B[3];
        locate(f, seed, c);
        orc_interp(f, f->b, c, seed, B);
        r->bn0 = B[0] * nrm[0] + B[1] * nrm[1] + B[2] * nrm[2];
    }
    if (!o->want_tw) r->tw = NAN;
    if (r->status & FATAL_BITS) r->tw = r->len = NAN;
    if (near_edge(f, r->face_b, r->end_b, o->edge_eps) ||
        near_edge(f, r->face_f, r->end_f, o->edge_eps))
        r->status |= ORC_EDGE;
}

static void trace_full(const orc_field *f, const double seed[3], const double nrm[3],
                       const orc_opts *o, double bnull2, full_line *r)
{
    trace_full_gen(f, seed, nrm, NULL, o, bnull2, r);
}

static void store_line(orc_lines *out, int64_t i, const full_line *r)
{
    if (!out) return;
    if (out->end_b) memcpy(out->end_b + 3 * i, r->end_b, 3 * sizeof(double));
    if (out->end_f) memcpy(out->end_f + 3 * i, r->end_f, 3 * sizeof(double));
    if (out->face_b) out->face_b[i] = (int8_t)r->face_b;
    if (out->face_f) out->face_f[i] = (int8_t)r->face_f;
    if (out->bn_b) out->bn_b[i] = r->bn_b;
    if (out->bn_f) out->bn_f[i] = r->bn_f;
    if (out->bn0) out->bn0[i] = r->bn0;
    if (out->tw) out->tw[i] = r->tw;
    if (out->len) out->len[i] = r->len;
    if (out->status) out->status[i] = (uint16_t)r->status;
    if (out->nsteps) out->nsteps[i] = r->nsteps;
}

static void set_threads(const orc_opts *o)
{
#ifdef _OPENMP
    if (o->nthreads > 0) omp_set_num_threads(o->nthreads);
#else
    (void)o;
#endif
}

int orc_trace(const orc_field *f, const double *seeds, int64_t n, const double *normal,
              const orc_opts *o, orc_lines *out)
{
    static const double zn[3] = {0.0, 0.0, 1.0};
    const double *nrm = normal ? normal : zn;
    double bnull2 = 1e-60 * field_scale2(f);
    set_threads(o);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < n; i++) {
        full_line r;
        trace_full(f, seeds + 3 * i, nrm, o, bnull2, &r);
        store_line(out, i, &r);
    }
    return 0;
}

/* ------------------------------------------------------------------------------
 * Method I squashing factor at one point of a seed grid
 * ---------------------------------------------------------------------------- */

/* One seed-grid axis of the Jacobian: derivatives of the in-face end coordinates
 * (u_b, v_b) and (u_f, v_f) with respect to the seed coordinate along the axis.
 * Central differences when both neighbours end on the centre line's faces at both
 * ends, else a one-sided difference with the neighbour that does; `m`/`p` are the
 * minus/plus neighbours (NULL where the grid ends). Returns 0 if no usable
 * neighbour exists. */
static int axis_jacobian(const full_line *c, const full_line *m, const full_line *p,
                         double delta, double d1[2], double d2[2], int *flags,
                         const orc_cyl *cyl)
{
    ends12 ec = order_ends(c);
    ends12 em = m ? order_ends(m) : ec, ep = p ? order_ends(p) : ec;
    int okm = m && !(m->status & FATAL_BITS) && em.f1 == ec.f1 && em.f2 == ec.f2;
    int okp = p && !(p->status & FATAL_BITS) && ep.f1 == ec.f1 && ep.f2 == ec.f2;
    double c1[2], c2[2], m1[2], m2[2], p1[2], p2[2];
    surf_uv(cyl, ec.f1, ec.e1, c1);
    surf_uv(cyl, ec.f2, ec.e2, c2);
    if (okm) {
        surf_uv(cyl, em.f1, em.e1, m1);
        surf_uv(cyl, em.f2, em.e2, m2);
        /* on the cylinder, arc lengths of neighbours are taken on the centre's branch */
        if (ec.f1 == ORC_FACE_CYL) m1[0] = unwrap(cyl, m1[0], c1[0]);
        if (ec.f2 == ORC_FACE_CYL) m2[0] = unwrap(cyl, m2[0], c2[0]);
    }
    if (okp) {
        surf_uv(cyl, ep.f1, ep.e1, p1);
        surf_uv(cyl, ep.f2, ep.e2, p2);
        if (ec.f1 == ORC_FACE_CYL) p1[0] = unwrap(cyl, p1[0], c1[0]);
        if (ec.f2 == ORC_FACE_CYL) p2[0] = unwrap(cyl, p2[0], c2[0]);
    }
    if (okm && okp) {
        for (int q = 0; q < 2; q++) {
            d1[q] = (p1[q] - m1[q]) / (2.0 * delta);
            d2[q] = (p2[q] - m2[q]) / (2.0 * delta);
        }
        return 1;
    }
    if (okp) {
        for (int q = 0; q < 2; q++) {
            d1[q] = (p1[q] - c1[q]) / delta;
            d2[q] = (p2[q] - c2[q]) / delta;
        }
        *flags |= ORC_ONESIDED;
        return 1;
    }
    if (okm) {
        for (int q = 0; q < 2; q++) {
            d1[q] = (c1[q] - m1[q]) / delta;
            d2[q] = (c2[q] - m2[q]) / delta;
        }
        *flags |= ORC_ONESIDED;
        return 1;
    }
    return 0;
}

/* Q at a point with centre line c, neighbours along the two S0 axes (x0, y0) and
 * spacings d0, d1. Eq. D+-2 and Eq. D+-3, then Eq. Q+- with |det D| -> |Bn1/Bn2|. */
static double method1_q(const full_line *c, const full_line *xm, const full_line *xp,
                        const full_line *ym, const full_line *yp, double d0, double d1,
                        double bn0, int *flags, const orc_cyl *cyl)
{
    double d1x[2], d2x[2], d1y[2], d2y[2];
    if (!axis_jacobian(c, xm, xp, d0, d1x, d2x, flags, cyl) ||
        !axis_jacobian(c, ym, yp, d1, d1y, d2y, flags, cyl)) {
        *flags |= ORC_MIXEDFACE;
        return NAN;
    }
    ends12 ec = order_ends(c);
    /* D10 = d(x1,y1)/d(x0,y0) */
    double dx1dx0 = d1x[0], dx1dy0 = d1y[0], dy1dx0 = d1x[1], dy1dy0 = d1y[1];
    /* D20 = d(x2,y2)/d(x0,y0) */
    double dx2dx0 = d2x[0], dx2dy0 = d2y[0], dy2dx0 = d2x[1], dy2dy0 = d2y[1];
    /* Eq. D+-3: (D10)^-1 = [[dy1/dy0, -dx1/dy0], [-dy1/dx0, dx1/dx0]] / |Bn0/Bn1| */
    double s = fabs(bn0 / ec.bn1);
    double i00 = dy1dy0 / s, i01 = -dx1dy0 / s, i10 = -dy1dx0 / s, i11 = dx1dx0 / s;
    /* Eq. D+-2: D12 = D20 (D10)^-1 */
    double a = dx2dx0 * i00 + dx2dy0 * i10;
    double b = dx2dx0 * i01 + dx2dy0 * i11;
    double cc = dy2dx0 * i00 + dy2dy0 * i10;
    double d = dy2dx0 * i01 + dy2dy0 * i11;
    /* Eq. Q+- with |det D12| -> |Bn1/Bn2| */
    return (a * a + b * b + cc * cc + d * d) / fabs(ec.bn1 / ec.bn2);
}

static void cross(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

static int on_box_face(const orc_field *f, const double r[3])
{
    for (int a = 0; a < 3; a++) {
        double tol = 1e-12 * mean_w(f, a);
        if (fabs(r[a] - box_lo(f, a)) <= tol || fabs(box_hi(f, a) - r[a]) <= tol) return 1;
    }
    return 0;
}

/* Section 4: where |Bn0/B| < 0.05 on an interior S0, rotate S0 perpendicular to the
 * line and trace four neighbours there, Bn0 becoming |B|. U = e_a x b / |..| with
 * e_a the axis least aligned with b, V = b x U. */
static double rotated_q(const orc_field *f, const double r0[3], const double B[3],
                        double delta, const full_line *c, const orc_opts *o, double bnull2,
                        int *flags)
{
    double bm = sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
    double bh[3] = {B[0] / bm, B[1] / bm, B[2] / bm};
    int a = 0;
    for (int q = 1; q < 3; q++)
        if (fabs(bh[q]) < fabs(bh[a])) a = q;
    double ea[3] = {0, 0, 0}, U[3], V[3];
    ea[a] = 1.0;
    cross(ea, bh, U);
    double um = sqrt(U[0] * U[0] + U[1] * U[1] + U[2] * U[2]);
    for (int q = 0; q < 3; q++) U[q] /= um;
    cross(bh, U, V);
    full_line nb[4];
    const double *dir[2] = {U, V};
    for (int ax = 0; ax < 2; ax++)
        for (int sgn = 0; sgn < 2; sgn++) {
            double s[3];
            double step = sgn ? delta : -delta;
            for (int q = 0; q < 3; q++) s[q] = r0[q] + step * dir[ax][q];
            trace_full(f, s, bh, o, bnull2, &nb[2 * ax + sgn]);
            if (nb[2 * ax + sgn].status & ORC_EDGE) *flags |= ORC_EDGE;
        }
    *flags |= ORC_ROTATED;
    return method1_q(c, &nb[0], &nb[1], &nb[2], &nb[3], delta, delta, bm, flags, NULL);
}

/* Q, Tw, length and status of one map point from its own line c and its stencil
 * neighbours (NULL where the grid ends); r0 is the seed, nrm the S0 normal. */
static void assemble_point(const orc_field *f, const full_line *c, const full_line *xm,
                           const full_line *xp, const full_line *ym, const full_line *yp,
                           const double r0[3], double du, double dv, const double nrm[3],
                           int allow_rotation, const orc_opts *o, double bnull2, double *q,
                           double *tw, double *len, uint16_t *status)
{
    int flags = c->status;
    double qv = NAN;
    if (!(c->status & FATAL_BITS)) {
        const full_line *nbs[4] = {xm, xp, ym, yp};
        double B[3];
        int64_t cl[3];
        locate(f, r0, cl);
        orc_interp(f, f->b, cl, r0, B);
        double bm = sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
        double bn0 = B[0] * nrm[0] + B[1] * nrm[1] + B[2] * nrm[2];
        if (allow_rotation && !on_box_face(f, r0) && fabs(bn0) < 0.05 * bm) {
            double delta = du < dv ? du : dv;
            qv = rotated_q(f, r0, B, delta, c, o, bnull2, &flags);
        } else {
            for (int k = 0; k < 4; k++)
                if (nbs[k] && (nbs[k]->status & ORC_EDGE)) flags |= ORC_EDGE;
            qv = method1_q(c, xm, xp, ym, yp, du, dv, bn0, &flags, NULL);
        }
    }
    *q = qv;
    *tw = c->tw;
    *len = c->len;
    *status = (uint16_t)flags;
}

/* Fill the map from traced lines on an nu x nv grid (i fastest). */
static void assemble_map(const orc_field *f, const full_line *lines, const double *seeds,
                         int64_t nu, int64_t nv, int64_t stride_layer, double du, double dv,
                         const double nrm[3], int allow_rotation, const orc_opts *o,
                         double bnull2, double *q, double *tw, double *len, uint16_t *status)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < nu * nv; p++) {
        int64_t i = p % nu, j = p / nu;
        int64_t idx = stride_layer + p;
        const full_line *c = &lines[idx];
        const full_line *xm = i > 0 ? &lines[idx - 1] : NULL;
        const full_line *xp = i < nu - 1 ? &lines[idx + 1] : NULL;
        const full_line *ym = j > 0 ? &lines[idx - nu] : NULL;
        const full_line *yp = j < nv - 1 ? &lines[idx + nu] : NULL;
        double qv, twv, lv;
        uint16_t sv;
        assemble_point(f, c, xm, xp, ym, yp, seeds + 3 * idx, du, dv, nrm, allow_rotation, o,
                       bnull2, &qv, &twv, &lv, &sv);
        if (q) q[idx] = qv;
        if (tw) tw[idx] = twv;
        if (len) len[idx] = lv;
        if (status) status[idx] = sv;
    }
}

/* Points of a layered map: point p = (i, j, k) -> seed base + i a + j b + k c, with
 * stencil neighbours along a and b inside an nu x nv layer. */
static int map_points(const orc_field *f, const double base[3], const double a[3],
                      const double b[3], const double c3[3], int64_t nu, int64_t nv,
                      int64_t nl, double du, double dv, const double nrm[3], const int64_t *pts,
                      int64_t npts, const orc_opts *o, double *q, double *tw, double *len,
                      uint16_t *status, orc_lines *lines_out)
{
    double bnull2 = 1e-60 * field_scale2(f);
    set_threads(o);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int64_t n = 0; n < npts; n++) {
        int64_t pt = pts[n];
        if (pt < 0 || pt >= nu * nv * nl) {
            bad = 1;
            continue;
        }
        int64_t k = pt / (nu * nv), r = pt % (nu * nv), j = r / nu, i = r % nu;
        /* centre, x-, x+, y-, y+ */
        const int64_t di[5] = {0, -1, 1, 0, 0}, dj[5] = {0, 0, 0, -1, 1};
        full_line L[5];
        int have[5];
        double seed0[3];
        for (int m = 0; m < 5; m++) {
            int64_t ii = i + di[m], jj = j + dj[m];
            have[m] = ii >= 0 && ii < nu && jj >= 0 && jj < nv;
            if (!have[m]) continue;
            double s[3];
            for (int e = 0; e < 3; e++)
                s[e] = base[e] + (double)ii * a[e] + (double)jj * b[e] + (double)k * c3[e];
            if (m == 0) memcpy(seed0, s, sizeof seed0);
            trace_full(f, s, nrm, o, bnull2, &L[m]);
        }
        double qv, twv, lv;
        uint16_t sv;
        assemble_point(f, &L[0], have[1] ? &L[1] : NULL, have[2] ? &L[2] : NULL,
                       have[3] ? &L[3] : NULL, have[4] ? &L[4] : NULL, seed0, du, dv, nrm, 1,
                       o, bnull2, &qv, &twv, &lv, &sv);
        if (q) q[n] = qv;
        if (tw) tw[n] = twv;
        if (len) len[n] = lv;
        if (status) status[n] = sv;
        if (lines_out) store_line(lines_out, n, &L[0]);
    }
    return bad ? -1 : 0;
}

int orc_q2d_points(const orc_field *f, const double origin[3], const double u[3],
                   const double v[3], int64_t nu, int64_t nv, double du, double dv,
                   const int64_t *pts, int64_t npts, const orc_opts *o, double *q, double *tw,
                   double *len, uint16_t *status, orc_lines *lines)
{
    double a[3], b[3], zero[3] = {0, 0, 0}, nrm[3];
    for (int e = 0; e < 3; e++) {
        a[e] = du * u[e];
        b[e] = dv * v[e];
    }
    cross(u, v, nrm);
    return map_points(f, origin, a, b, zero, nu, nv, 1, du, dv, nrm, pts, npts, o, q, tw, len,
                      status, lines);
}

int orc_q3d_points(const orc_field *f, const double origin[3], const double spacing[3],
                   const int64_t nvox[3], const int64_t *pts, int64_t npts, const orc_opts *o,
                   double *q, double *tw, double *len, uint16_t *status, orc_lines *lines)
{
    const double a[3] = {spacing[0], 0, 0}, b[3] = {0, spacing[1], 0}, c3[3] = {0, 0, spacing[2]};
    const double nrm[3] = {0.0, 0.0, 1.0};
    return map_points(f, origin, a, b, c3, nvox[0], nvox[1], nvox[2], spacing[0], spacing[1],
                      nrm, pts, npts, o, q, tw, len, status, lines);
}

int orc_q2d(const orc_field *f, const double origin[3], const double u[3],
            const double v[3], int64_t nu, int64_t nv, double du, double dv,
            const orc_opts *o, double *q, double *tw, double *len, uint16_t *status,
            orc_lines *lines_out)
{
    if (nu < 1 || nv < 1) return -1;
    set_threads(o);
    int64_t n = nu * nv;
    double *seeds = (double *)malloc((size_t)n * 3 * sizeof(double));
    full_line *lines = (full_line *)malloc((size_t)n * sizeof(full_line));
    if (!seeds || !lines) {
        free(seeds);
        free(lines);
        return -2;
    }
    for (int64_t j = 0; j < nv; j++)
        for (int64_t i = 0; i < nu; i++)
            for (int a = 0; a < 3; a++)
                seeds[3 * (j * nu + i) + a] =
                    origin[a] + (double)i * du * u[a] + (double)j * dv * v[a];
    double nrm[3];
    cross(u, v, nrm);
    double bnull2 = 1e-60 * field_scale2(f);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < n; i++) trace_full(f, seeds + 3 * i, nrm, o, bnull2, &lines[i]);
    assemble_map(f, lines, seeds, nu, nv, 0, du, dv, nrm, 1, o, bnull2, q, tw, len, status);
    if (lines_out)
        for (int64_t i = 0; i < n; i++) store_line(lines_out, i, &lines[i]);
    free(seeds);
    free(lines);
    return 0;
}

int orc_q3d(const orc_field *f, const double origin[3], const double spacing[3],
            const int64_t nvox[3], const orc_opts *o, double *q, double *tw, double *len,
            uint16_t *status, orc_lines *lines_out)
{
    if (nvox[0] < 1 || nvox[1] < 1 || nvox[2] < 1) return -1;
    set_threads(o);
    int64_t layer = nvox[0] * nvox[1];
    int64_t n = layer * nvox[2];
    double *seeds = (double *)malloc((size_t)n * 3 * sizeof(double));
    full_line *lines = (full_line *)malloc((size_t)n * sizeof(full_line));
    if (!seeds || !lines) {
        free(seeds);
        free(lines);
        return -2;
    }
    for (int64_t k = 0; k < nvox[2]; k++)
        for (int64_t j = 0; j < nvox[1]; j++)
            for (int64_t i = 0; i < nvox[0]; i++) {
                int64_t p = (k * nvox[1] + j) * nvox[0] + i;
                seeds[3 * p + 0] = origin[0] + (double)i * spacing[0];
                seeds[3 * p + 1] = origin[1] + (double)j * spacing[1];
                seeds[3 * p + 2] = origin[2] + (double)k * spacing[2];
            }
    const double nrm[3] = {0.0, 0.0, 1.0};
    double bnull2 = 1e-60 * field_scale2(f);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < n; i++) trace_full(f, seeds + 3 * i, nrm, o, bnull2, &lines[i]);
    for (int64_t k = 0; k < nvox[2]; k++)
        assemble_map(f, lines, seeds, nvox[0], nvox[1], k * layer, spacing[0], spacing[1],
                     nrm, 1, o, bnull2, q, tw, len, status);
    if (lines_out)
        for (int64_t i = 0; i < n; i++) store_line(lines_out, i, &lines[i]);
    free(seeds);
    free(lines);
    return 0;
}

/* ------------------------------------------------------------------------------
 * A cylindrical mapping surface (Section 3, the x^2 + y^2 = 1 example)
 * ---------------------------------------------------------------------------- */

int orc_qcyl(const orc_field *f, const orc_cyl *cyl, double theta0, double dtheta,
             int64_t ntheta, double z0, double dz, int64_t nz, const orc_opts *o, double *q,
             double *tw, double *len, uint16_t *status, orc_lines *lines_out)
{
    if (ntheta < 1 || nz < 1 || !(cyl->r > 0.0)) return -1;
    set_threads(o);
    int64_t n = ntheta * nz;
    double *seeds = (double *)malloc((size_t)n * 3 * sizeof(double));
    full_line *lines = (full_line *)malloc((size_t)n * sizeof(full_line));
    if (!seeds || !lines) {
        free(seeds);
        free(lines);
        return -2;
    }
    for (int64_t j = 0; j < nz; j++)
        for (int64_t i = 0; i < ntheta; i++) {
            double th = theta0 + (double)i * dtheta;
            double *s3 = seeds + 3 * (j * ntheta + i);
            s3[0] = cyl->xc + cyl->r * cos(th);
            s3[1] = cyl->yc + cyl->r * sin(th);
            s3[2] = z0 + (double)j * dz;
        }
    double bnull2 = 1e-60 * field_scale2(f);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < n; i++) {
        double nrm[3];
        cyl_normal(cyl, seeds + 3 * i, nrm);
        trace_full_gen(f, seeds + 3 * i, nrm, cyl, o, bnull2, &lines[i]);
    }
    /* Method I on S0 = the cylinder (coordinates r theta, z; neighbours along theta
     * and z), S1 = the seed's own end, S2 = where the line meets the cylinder again
     * (or a box face) */
    double d0 = cyl->r * dtheta;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < n; p++) {
        int64_t i = p % ntheta, j = p / ntheta;
        const full_line *c = &lines[p];
        const full_line *xm = i > 0 ? &lines[p - 1] : NULL;
        const full_line *xp = i < ntheta - 1 ? &lines[p + 1] : NULL;
        const full_line *ym = j > 0 ? &lines[p - ntheta] : NULL;
        const full_line *yp = j < nz - 1 ? &lines[p + ntheta] : NULL;
        int flags = c->status;
        double qv = NAN;
        if (!(c->status & FATAL_BITS)) {
            const full_line *nbs[4] = {xm, xp, ym, yp};
            for (int k = 0; k < 4; k++)
                if (nbs[k] && (nbs[k]->status & ORC_EDGE)) flags |= ORC_EDGE;
            qv = method1_q(c, xm, xp, ym, yp, d0, dz, c->bn0, &flags, cyl);
        }
        if (q) q[p] = qv;
        if (tw) tw[p] = c->tw;
        if (len) len[p] = c->len;
        if (status) status[p] = (uint16_t)flags;
        if (lines_out) store_line(lines_out, p, c);
    }
    free(seeds);
    free(lines);
    return 0;
}

/* ------------------------------------------------------------------------------
 * Method I with S1, S2 perpendicular to B at the ends (Q_perp, Section 2.1), and the
 * field-line length edge map
 * ---------------------------------------------------------------------------- */

/* One S0 axis of the 3-D end Jacobians: derivatives of the S1 and S2 end points with
 * respect to the seed coordinate along the axis, by the stencil rule of
 * axis_jacobian (central where both neighbours end on the centre line's faces,
 * else one-sided), and the same derivative of the line length. Returns 0 if no
 * neighbour is usable. */
static int axis_jacobian3(const full_line *c, const full_line *m, const full_line *p,
                          double delta, double j1[3], double j2[3], double *dl)
{
    ends12 ec = order_ends(c);
    ends12 em = m ? order_ends(m) : ec, ep = p ? order_ends(p) : ec;
    int okm = m && !(m->status & FATAL_BITS) && em.f1 == ec.f1 && em.f2 == ec.f2;
    int okp = p && !(p->status & FATAL_BITS) && ep.f1 == ec.f1 && ep.f2 == ec.f2;
    const full_line *lo = okm ? m : c, *hi = okp ? p : c;
    ends12 el = okm ? em : ec, eh = okp ? ep : ec;
    if (!okm && !okp) return 0;
    double span = (okm && okp) ? 2.0 * delta : delta;
    for (int q = 0; q < 3; q++) {
        j1[q] = (eh.e1[q] - el.e1[q]) / span;
        j2[q] = (eh.e2[q] - el.e2[q]) / span;
    }
    *dl = (hi->len - lo->len) / span;
    return 1;
}

static double dot3(const double a[3], const double b[3]);

/* v minus its component along the unit vector b. */
static void perp_to(const double v[3], const double b[3], double out[3])
{
    double t = v[0] * b[0] + v[1] * b[1] + v[2] * b[2];
    for (int q = 0; q < 3; q++) out[q] = v[q] - t * b[q];
}

/* Q_perp at a point (Section 2.1: S1, S2 rotated perpendicular to the line at its
 * ends). The end displacements of neighbouring lines, projected along B onto the
 * planes perpendicular to B at the ends, give the maps from S0 to S1_perp and to
 * S2_perp, with Gram matrices G1, G2 (2 x 2). The map S1_perp -> S2_perp has squared
 * norm tr(G1^-1 G2); its determinant is |B1/B2| (flux through perpendicular
 * sections), and the inverse of G1 is written, as in Eq. D+-3, with its determinant
 * from the flux through S0: det G1 = (Bn0/|B1|)^2. So Q_perp = tr(adj(G1) G2)
 * |B1| |B2| / Bn0^2. Also |grad_S0 length| (the length edge map). */
static void method1_perp(const orc_field *f, const full_line *c, const full_line *xm,
                         const full_line *xp, const full_line *ym, const full_line *yp,
                         double d0, double d1, double bn0, double *qperp, double *fledge,
                         int *flags)
{
    double j1x[3], j2x[3], j1y[3], j2y[3], dlx, dly;
    *qperp = *fledge = NAN;
    if (!axis_jacobian3(c, xm, xp, d0, j1x, j2x, &dlx) ||
        !axis_jacobian3(c, ym, yp, d1, j1y, j2y, &dly)) {
        *flags |= ORC_MIXEDFACE;
        return;
    }
    *fledge = sqrt(dlx * dlx + dly * dly);
    ends12 ec = order_ends(c);
    double B1[3], B2[3], b1[3], b2[3];
    int64_t cl[3];
    locate(f, ec.e1, cl);
    orc_interp(f, f->b, cl, ec.e1, B1);
    locate(f, ec.e2, cl);
    orc_interp(f, f->b, cl, ec.e2, B2);
    double m1 = sqrt(B1[0] * B1[0] + B1[1] * B1[1] + B1[2] * B1[2]);
    double m2 = sqrt(B2[0] * B2[0] + B2[1] * B2[1] + B2[2] * B2[2]);
    for (int q = 0; q < 3; q++) {
        b1[q] = B1[q] / m1;
        b2[q] = B2[q] / m2;
    }
    double p1x[3], p1y[3], p2x[3], p2y[3];
    perp_to(j1x, b1, p1x);
    perp_to(j1y, b1, p1y);
    perp_to(j2x, b2, p2x);
    perp_to(j2y, b2, p2y);
    /* G1 = [[g11, g12], [g12, g22]], adj(G1) = [[g22, -g12], [-g12, g11]] */
    double g11 = dot3(p1x, p1x), g12 = dot3(p1x, p1y), g22 = dot3(p1y, p1y);
    double h11 = dot3(p2x, p2x), h12 = dot3(p2x, p2y), h22 = dot3(p2y, p2y);
    double tr = g22 * h11 - 2.0 * g12 * h12 + g11 * h22;
    *qperp = tr * m1 * m2 / (bn0 * bn0);
}

int orc_q2d_perp(const orc_field *f, const double origin[3], const double u[3],
                 const double v[3], int64_t nu, int64_t nv, double du, double dv,
                 const orc_opts *o, double *qperp, double *fledge, uint16_t *status)
{
    if (nu < 1 || nv < 1) return -1;
    set_threads(o);
    int64_t n = nu * nv;
    double *seeds = (double *)malloc((size_t)n * 3 * sizeof(double));
    full_line *lines = (full_line *)malloc((size_t)n * sizeof(full_line));
    if (!seeds || !lines) {
        free(seeds);
        free(lines);
        return -2;
    }
    for (int64_t j = 0; j < nv; j++)
        for (int64_t i = 0; i < nu; i++)
            for (int a = 0; a < 3; a++)
                seeds[3 * (j * nu + i) + a] =
                    origin[a] + (double)i * du * u[a] + (double)j * dv * v[a];
    double nrm[3];
    cross(u, v, nrm);
    double bnull2 = 1e-60 * field_scale2(f);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < n; i++) trace_full(f, seeds + 3 * i, nrm, o, bnull2, &lines[i]);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < n; p++) {
        int64_t i = p % nu, j = p / nu;
        const full_line *c = &lines[p];
        const full_line *xm = i > 0 ? &lines[p - 1] : NULL;
        const full_line *xp = i < nu - 1 ? &lines[p + 1] : NULL;
        const full_line *ym = j > 0 ? &lines[p - nu] : NULL;
        const full_line *yp = j < nv - 1 ? &lines[p + nu] : NULL;
        int flags = c->status;
        double qp = NAN, fl = NAN;
        const double *r0 = seeds + 3 * p;
        if (!(c->status & FATAL_BITS)) {
            double B[3];
            int64_t cl[3];
            locate(f, r0, cl);
            orc_interp(f, f->b, cl, r0, B);
            double bm = sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
            double bn0 = B[0] * nrm[0] + B[1] * nrm[1] + B[2] * nrm[2];
            const full_line *nbs[4] = {xm, xp, ym, yp};
            for (int k = 0; k < 4; k++)
                if (nbs[k] && (nbs[k]->status & ORC_EDGE)) flags |= ORC_EDGE;
            if (!on_box_face(f, r0) && fabs(bn0) < 0.05 * bm) flags |= ORC_ROTATED; /* not formed */
            else method1_perp(f, c, xm, xp, ym, yp, du, dv, bn0, &qp, &fl, &flags);
        }
        if (qperp) qperp[p] = qp;
        if (fledge) fledge[p] = fl;
        if (status) status[p] = (uint16_t)flags;
    }
    free(seeds);
    free(lines);
    return 0;
}

/* ------------------------------------------------------------------------------
 * Method II (Section 2.1, Eq. rb2 and Eq. q_scott)
 * ---------------------------------------------------------------------------- */

/* Components of the node array of grad(B/B) (Section 4, Eq. grad_B): plane 3 i + j
 * holds d(B_i/B)/dx_j at every node, by the same second-order differences as the
 * curl (central inside, one-sided on boundary nodes), applied to B/B. */
static int grad_b_planes(const orc_field *f, double *planes[9])
{
    int64_t nn = f->n[0] * f->n[1] * f->n[2];
    double *u[3];
    for (int a = 0; a < 3; a++) {
        u[a] = (double *)malloc((size_t)nn * sizeof(double));
        if (!u[a]) {
            for (int b = 0; b < a; b++) free(u[b]);
            return -2;
        }
    }
    for (int64_t q = 0; q < nn; q++) {
        double bm = sqrt(f->b[0][q] * f->b[0][q] + f->b[1][q] * f->b[1][q] + f->b[2][q] * f->b[2][q]);
        for (int a = 0; a < 3; a++) u[a][q] = bm > 0.0 ? f->b[a][q] / bm : 0.0;
    }
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t k = 0; k < f->n[2]; k++)
        for (int64_t j = 0; j < f->n[1]; j++)
            for (int64_t i = 0; i < f->n[0]; i++) {
                int64_t q = node(f, i, j, k);
                for (int c = 0; c < 3; c++)
                    for (int ax = 0; ax < 3; ax++)
                        planes[3 * c + ax][q] = deriv(f, u[c], ax, i, j, k);
            }
    for (int a = 0; a < 3; a++) free(u[a]);
    return 0;
}

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* The two ends' tangent vectors moved onto their end planes along B:
 * W~ = W - (W . n) / (B . n) B, with n the plane's normal. */
static void project_along_b(const double W[3], const double n[3], const double B[3], double out[3])
{
    double s = dot3(W, n) / dot3(B, n);
    for (int a = 0; a < 3; a++) out[a] = W[a] - s * B[a];
}

/* Eq. q_scott's numerator for projected tangent vectors (U1, V1) and (U2, V2). */
static double scott_num(const double U1[3], const double V1[3], const double U2[3],
                        const double V2[3])
{
    return dot3(U1, U1) * dot3(V2, V2) + dot3(U2, U2) * dot3(V1, V1) -
           2.0 * dot3(U1, V1) * dot3(U2, V2);
}

int orc_method2(const orc_field *f, const double *seeds, int64_t n, int way, const orc_opts *o,
                double *q, double *qperp, double *tw, double *len, uint16_t *status,
                orc_lines *out)
{
    if (way != 1 && way != 2) return -1;
    double *gp[9] = {NULL};
    if (way == 1) {
        int64_t nn = f->n[0] * f->n[1] * f->n[2];
        for (int a = 0; a < 9; a++) {
            gp[a] = (double *)malloc((size_t)nn * sizeof(double));
            if (!gp[a]) {
                for (int b = 0; b < a; b++) free(gp[b]);
                return -2;
            }
        }
        if (grad_b_planes(f, gp)) {
            for (int a = 0; a < 9; a++) free(gp[a]);
            return -2;
        }
    }
    double bnull2 = 1e-60 * field_scale2(f);
    set_threads(o);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < n; i++) {
        const double *r0 = seeds + 3 * i;
        full_line r;
        memset(&r, 0, sizeof r);
        double qv = NAN, qp = NAN;
        int flags = 0;
        half_line hb, hf;
        if (!in_box(f, r0)) {
            flags = ORC_OUTSIDE;
            hb.face = hf.face = -1;
        } else {
            /* S0 perpendicular to B at the seed (Section 4: Method II always takes the
             * perpendicular S0), U and V orthonormal in it: U = e_a x b / |..| with e_a
             * the axis least aligned with b, V = b x U */
            int64_t c[3];
            double B0[3];
            locate(f, r0, c);
            orc_interp(f, f->b, c, r0, B0);
            double bm0 = sqrt(dot3(B0, B0));
            m2_ctx m;
            m.way = way;
            m.gb = (const double *const *)gp;
            if (!(bm0 * bm0 > bnull2)) {
                flags = ORC_NULLB;
                hb.face = hf.face = -1;
            } else {
                double bh[3] = {B0[0] / bm0, B0[1] / bm0, B0[2] / bm0};
                int a = 0;
                for (int k = 1; k < 3; k++)
                    if (fabs(bh[k]) < fabs(bh[a])) a = k;
                double ea[3] = {0, 0, 0};
                ea[a] = 1.0;
                cross(ea, bh, m.U0);
                double um = sqrt(dot3(m.U0, m.U0));
                for (int k = 0; k < 3; k++) m.U0[k] /= um;
                cross(bh, m.U0, m.V0);
                trace_half_gen(f, r0, -1, o, bnull2, &m, NULL, &hb);
                trace_half_gen(f, r0, +1, o, bnull2, &m, NULL, &hf);
                flags = hb.status | hf.status;
                if (!(flags & FATAL_BITS)) {
                    /* Eq. q_scott with S1, S2 the faces the line ends on ... */
                    double n1[3] = {0, 0, 0}, n2[3] = {0, 0, 0}, B1[3], B2[3];
                    int64_t c1[3], c2[3];
                    n1[hb.face / 2] = 1.0;
                    n2[hf.face / 2] = 1.0;
                    locate(f, hb.end, c1);
                    locate(f, hf.end, c2);
                    orc_interp(f, f->b, c1, hb.end, B1);
                    orc_interp(f, f->b, c2, hf.end, B2);
                    double U1[3], V1[3], U2[3], V2[3];
                    project_along_b(hb.U, n1, B1, U1);
                    project_along_b(hb.V, n1, B1, V1);
                    project_along_b(hf.U, n2, B2, U2);
                    project_along_b(hf.V, n2, B2, V2);
                    qv = scott_num(U1, V1, U2, V2) * fabs(dot3(B1, n1) * dot3(B2, n2)) /
                         (bm0 * bm0);
                    /* ... and with S1, S2 perpendicular to B at the ends (Q_perp) */
                    double b1m = sqrt(dot3(B1, B1)), b2m = sqrt(dot3(B2, B2));
                    double t1[3] = {B1[0] / b1m, B1[1] / b1m, B1[2] / b1m};
                    double t2[3] = {B2[0] / b2m, B2[1] / b2m, B2[2] / b2m};
                    project_along_b(hb.U, t1, B1, U1);
                    project_along_b(hb.V, t1, B1, V1);
                    project_along_b(hf.U, t2, B2, U2);
                    project_along_b(hf.V, t2, B2, V2);
                    qp = scott_num(U1, V1, U2, V2) * b1m * b2m / (bm0 * bm0);
                }
                if (near_edge(f, hb.face, hb.end, o->edge_eps) ||
                    near_edge(f, hf.face, hf.end, o->edge_eps))
                    flags |= ORC_EDGE;
            }
        }
        if (q) q[i] = qv;
        if (qperp) qperp[i] = qp;
        int fatal = (flags & FATAL_BITS) != 0;
        if (tw) tw[i] = (fatal || !o->want_tw) ? NAN : hb.tw + hf.tw;
        if (len) len[i] = fatal ? NAN : hb.len + hf.len;
        if (status) status[i] = (uint16_t)flags;
        if (out) {
            if (out->end_b) memcpy(out->end_b + 3 * i, fatal ? (double[3]){NAN, NAN, NAN} : hb.end, 3 * sizeof(double));
            if (out->end_f) memcpy(out->end_f + 3 * i, fatal ? (double[3]){NAN, NAN, NAN} : hf.end, 3 * sizeof(double));
            if (out->face_b) out->face_b[i] = (int8_t)(fatal ? -1 : hb.face);
            if (out->face_f) out->face_f[i] = (int8_t)(fatal ? -1 : hf.face);
            if (out->status) out->status[i] = (uint16_t)flags;
        }
        (void)r;
    }
    for (int a = 0; a < 9; a++) free(gp[a]);
    return 0;
}
