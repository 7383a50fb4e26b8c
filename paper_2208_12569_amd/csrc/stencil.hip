// Method-I map assembly in FP64.
//
// From the traced half lines, each map point gets the Jacobians of both end maps by
// differences over its neighbouring seeds and Q = (a^2+b^2+c^2+d^2)/|Bn1/Bn2| with
// D12 = D20 (D10)^-1 (Section 2.1, Eq. D+-2 and Eq. D+-3; Section 1, Eq. Q+- and
// Eq. Bn1). Written as Q = ||J2 adj(J1)||_F^2 |Bn1 Bn2| / Bn0^2, which is the same
// quantity: (D10)^-1 = adj(J1) / |Bn0/Bn1| and |det D12| -> |Bn1/Bn2|.
//
// Every normal field Bn0, Bn1, Bn2 is interpolated in FP64 from the caller's planes
// (the FP64 fix-up of the FP32 form): a near-tangent seed has |Bn0| << |B| and an
// FP32 value would cost Q its accuracy there.
//
// Stencil rule: central differences along an S0 axis where both neighbours end on
// the centre line's faces at both ends; else a one-sided difference with the
// neighbour that does (FQ_ST_ONESIDED); else Q = NaN (FQ_ST_MIXEDFACE, the case
// Code2016 returns NaN for, Section 2.1). For a seed on a box face one half line
// has zero length and ends at the seed; that end is taken as S1, whatever the
// polarity, so that seeds on both sides of a polarity inversion line difference the
// same seed -> far-footpoint map.
#include <math.h>

#include "fq_internal.h"
#include "stencil_dev.h"

namespace fq {
namespace {

using namespace sten;

// Q from the centre line and its four S0 neighbours (present flags hxm..hyp).
__device__ __forceinline__ double q_nb(const MapJob &m, const Line &c, const Nb &xm, bool hxm,
                                       const Nb &xp, bool hxp, const Nb &ym, bool hym, const Nb &yp,
                                       bool hyp, double d0, double d1, double bn0, uint16_t &st)
{
    double c1[2], c2[2];
    inface(c.f1, c.e1, c1);
    inface(c.f2, c.e2, c2);
    // axis by axis, so that a one-sided x difference is flagged also where y fails
    double ax1[2], ax2[2], ay1[2], ay2[2];
    const int rx = axis_rule(c, xm, hxm, xp, hxp);
    if (rx != RULE_NONE) axis_diff(rx, c1, c2, xm, xp, d0, ax1, ax2, st);
    const int ry = rx == RULE_NONE ? RULE_NONE : axis_rule(c, ym, hym, yp, hyp);
    if (ry == RULE_NONE) {
        st |= FQ_ST_MIXEDFACE;
        return NAN;
    }
    axis_diff(ry, c1, c2, ym, yp, d1, ay1, ay2, st);
    // J1 = [[du1/dx0, du1/dy0], [dv1/dx0, dv1/dy0]], likewise J2
    const double j00 = ax1[0], j01 = ay1[0], j10 = ax1[1], j11 = ay1[1];
    const double k00 = ax2[0], k01 = ay2[0], k10 = ax2[1], k11 = ay2[1];
    // M = J2 adj(J1), adj(J1) = [[j11, -j01], [-j10, j00]]
    const double m00 = k00 * j11 - k01 * j10;
    const double m01 = -k00 * j01 + k01 * j00;
    const double m10 = k10 * j11 - k11 * j10;
    const double m11 = -k10 * j01 + k11 * j00;
    double B1[3], B2[3];
    field64(m, c.e1, B1);
    field64(m, c.e2, B2);
    const double bn1 = comp3(B1, c.f1 >> 1), bn2 = comp3(B2, c.f2 >> 1);
    const double nrm = m00 * m00 + m01 * m01 + m10 * m10 + m11 * m11;
    return nrm * fabs(bn1 * bn2) / (bn0 * bn0);
}

__device__ __forceinline__ bool on_box_face(const MapJob &m, const double r[3])
{
    for (int a = 0; a < 3; a++) {
        const double tol = 1e-12 * axis_width(m, a);
        const double lo = axis_lo(m, a), hi = axis_hi(m, a);
        if (fabs(r[a] - lo) <= tol || fabs(hi - r[a]) <= tol) return true;
    }
    return false;
}

__global__ void classify_kernel(MapJob m, int32_t *rot_index, RotEntry *rot,
                                uint32_t *rot_count, int64_t capacity)
{
    const int64_t lay = m.nu * m.nv, np = lay * m.nlayers;
    for (int64_t pt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pt < np;
         pt += (int64_t)gridDim.x * blockDim.x) {
        int32_t idx = -1;
        const int64_t k = pt / lay, r2 = pt - k * lay, j = r2 / m.nu, i = r2 - j * m.nu;
        double r[3];
        point_pos(m, i, j, k, r);
        bool inside = true;
        for (int a = 0; a < 3; a++) {
            const double lo = axis_lo(m, a), hi = axis_hi(m, a);
            if (!(r[a] >= lo && r[a] <= hi)) inside = false;
        }
        if (inside && !on_box_face(m, r)) {
            double B[3];
            field64(m, r, B);
            const double bm = sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
            const double bn = B[0] * m.normal[0] + B[1] * m.normal[1] + B[2] * m.normal[2];
            if (bm > 0.0 && fabs(bn) < 0.05 * bm) {
                // Section 4: rotate S0 perpendicular to the line
                const double b[3] = {B[0] / bm, B[1] / bm, B[2] / bm};
                int a = 0;
                if (fabs(b[1]) < fabs(b[a])) a = 1;
                if (fabs(b[2]) < fabs(b[a])) a = 2;
                double ea[3] = {0.0, 0.0, 0.0};
                ea[a] = 1.0;
                double U[3] = {ea[1] * b[2] - ea[2] * b[1], ea[2] * b[0] - ea[0] * b[2],
                               ea[0] * b[1] - ea[1] * b[0]};
                const double un = sqrt(U[0] * U[0] + U[1] * U[1] + U[2] * U[2]);
                for (int q = 0; q < 3; q++) U[q] /= un;
                const double V[3] = {b[1] * U[2] - b[2] * U[1], b[2] * U[0] - b[0] * U[2],
                                     b[0] * U[1] - b[1] * U[0]};
                const uint32_t slot = atomicAdd(rot_count, 1u);
                if ((int64_t)slot < capacity) {
                    RotEntry &e = rot[slot];
                    e.point = pt;
                    for (int q = 0; q < 3; q++) {
                        e.r0[q] = r[q];
                        e.U[q] = U[q];
                        e.V[q] = V[q];
                    }
                    idx = (int32_t)slot;
                } else {
                    idx = -2;  // over capacity: no Q at this point
                }
            }
        }
        rot_index[pt] = idx;
    }
}

// The normal field at an end on `face`: the face's axis component, or on a
// cylindrical mapping surface the component along its outward normal.
__device__ __forceinline__ double end_bn(const MapJob &m, int face, const double e[3], const double B[3])
{
    if (face == kFaceCyl) {
        const double dx = e[0] - m.cyl[0], dy = e[1] - m.cyl[1];
        return (B[0] * dx + B[1] * dy) / sqrt(dx * dx + dy * dy);
    }
    return comp3(B, face >> 1);
}

__device__ __forceinline__ void write_line(const MapJob &m, const fq_lines &o, int64_t l, const double seed[3])
{
    const int64_t hb = l, hf = m.nlines + l;
    uint16_t st = m.rec.st[hb] | m.rec.st[hf];
    double eb[3], ef[3];
    for (int a = 0; a < 3; a++) {
        eb[a] = m.rec.end[3 * hb + a];
        ef[a] = m.rec.end[3 * hf + a];
    }
    const int fb = m.rec.face[hb], ff = m.rec.face[hf];
    if (edge_end(m, fb, eb) || edge_end(m, ff, ef)) st |= FQ_ST_EDGE;
    const bool bad = (st & kFatal) != 0;
    if (o.end_b)
        for (int a = 0; a < 3; a++) o.end_b[3 * l + a] = eb[a];
    if (o.end_f)
        for (int a = 0; a < 3; a++) o.end_f[3 * l + a] = ef[a];
    if (o.face_b) o.face_b[l] = (int8_t)fb;
    if (o.face_f) o.face_f[l] = (int8_t)ff;
    if (o.bn_b || o.bn_f || o.bn0) {
        double B[3];
        if (o.bn_b) {
            if (fb >= 0) {
                field64(m, eb, B);
                o.bn_b[l] = end_bn(m, fb, eb, B);
            } else o.bn_b[l] = NAN;
        }
        if (o.bn_f) {
            if (ff >= 0) {
                field64(m, ef, B);
                o.bn_f[l] = end_bn(m, ff, ef, B);
            } else o.bn_f[l] = NAN;
        }
        if (o.bn0) {
            if (st & FQ_ST_OUTSIDE) o.bn0[l] = NAN;
            else {
                field64(m, seed, B);
                o.bn0[l] = m.is_cyl ? end_bn(m, kFaceCyl, seed, B)
                                    : B[0] * m.normal[0] + B[1] * m.normal[1] + B[2] * m.normal[2];
            }
        }
    }
    if (o.tw) o.tw[l] = bad ? NAN : m.rec.tw[hb] + m.rec.tw[hf];
    if (o.length) o.length[l] = bad ? NAN : m.rec.len[hb] + m.rec.len[hf];
    if (o.status) o.status[l] = st;
}

__global__ __launch_bounds__(256) void stencil_kernel(MapJob m)
{
    const int64_t lay = m.nu * m.nv, np = lay * m.nlayers;
    for (int64_t pt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pt < np;
         pt += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = pt / lay, r2 = pt - k * lay, j = r2 / m.nu, i = r2 - j * m.nu;
        double r0[3];
        point_pos(m, i, j, k, r0);
        Line c;
        read_line(m.rec, m.nlines, pt, c);
        uint16_t st = c.st;
        if (edge_end(m, c.f1, c.e1) || edge_end(m, c.f2, c.e2)) st |= FQ_ST_EDGE;
        double q = NAN, tw = NAN, len = NAN;
        if (!(c.st & kFatal)) {
            tw = c.tw;
            len = c.len;
            const int32_t ri = m.rot_index ? m.rot_index[pt] : -1;
            if (ri >= 0) {
                const int64_t r4 = 4 * (int64_t)ri;
                const Nb n0 = read_nb(m, m.rot_rec, m.rot_nlines, r4 + 0);
                const Nb n1 = read_nb(m, m.rot_rec, m.rot_nlines, r4 + 1);
                const Nb n2 = read_nb(m, m.rot_rec, m.rot_nlines, r4 + 2);
                const Nb n3 = read_nb(m, m.rot_rec, m.rot_nlines, r4 + 3);
                if (n0.edge || n1.edge || n2.edge || n3.edge) st |= FQ_ST_EDGE;
                double B[3];
                field64(m, r0, B);
                const double bm = sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
                st |= FQ_ST_ROTATED;
                q = q_nb(m, c, n0, true, n1, true, n2, true, n3, true, m.rot_delta, m.rot_delta, bm, st);
            } else if (ri == -2) {
                st |= FQ_ST_ROTATED | FQ_ST_MIXEDFACE;
            } else {
                const bool hxm = i > 0, hxp = i < m.nu - 1, hym = j > 0, hyp = j < m.nv - 1;
                // a missing neighbour reads the centre's own record (never used)
                const Nb xm = read_nb(m, m.rec, m.nlines, hxm ? pt - 1 : pt);
                const Nb xp = read_nb(m, m.rec, m.nlines, hxp ? pt + 1 : pt);
                const Nb ym = read_nb(m, m.rec, m.nlines, hym ? pt - m.nu : pt);
                const Nb yp = read_nb(m, m.rec, m.nlines, hyp ? pt + m.nu : pt);
                if ((hxm && xm.edge) || (hxp && xp.edge) || (hym && ym.edge) || (hyp && yp.edge))
                    st |= FQ_ST_EDGE;
                double B[3];
                field64(m, r0, B);
                const double bn0 = B[0] * m.normal[0] + B[1] * m.normal[1] + B[2] * m.normal[2];
                q = q_nb(m, c, xm, hxm, xp, hxp, ym, hym, yp, hyp, m.d0, m.d1, bn0, st);
            }
        }
        if (m.out.q) m.out.q[pt] = q;
        if (m.out.tw) m.out.tw[pt] = tw;
        if (m.out.length) m.out.length[pt] = len;
        if (m.out.status) m.out.status[pt] = st;
        const fq_lines &o = m.out.lines;
        if (o.end_b || o.end_f || o.face_b || o.face_f || o.bn_b || o.bn_f || o.bn0 || o.tw ||
            o.length || o.status)
            write_line(m, o, pt, r0);
    }
}

// Method II (Section 2.1, Eq. q_scott): the tangent vectors at each end, moved onto
// the end's plane along B, W~ = W - (W . n) / (B . n) B, give
// Q = (U1~^2 V2~^2 + U2~^2 V1~^2 - 2 (U1~ . V1~)(U2~ . V2~)) |Bn1 Bn2| / Bn0^2 with S1, S2
// the faces the line ends on, and Q_perp with n = B/|B| at each end (planes
// perpendicular to B, Bn = |B|). S0 is perpendicular to B at the seed: Bn0 = |B0|.
__device__ __forceinline__ double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

__device__ __forceinline__ void along_b(const double W[3], const double n[3], const double B[3],
                                        double o[3])
{
    const double t = dot3(W, n) / dot3(B, n);
    for (int a = 0; a < 3; a++) o[a] = W[a] - t * B[a];
}

__device__ __forceinline__ double scott(const double U1[3], const double V1[3], const double U2[3],
                                        const double V2[3])
{
    return dot3(U1, U1) * dot3(V2, V2) + dot3(U2, U2) * dot3(V1, V1) -
           2.0 * dot3(U1, V1) * dot3(U2, V2);
}

__global__ __launch_bounds__(256) void m2_map_kernel(MapJob m)
{
    const int64_t lay = m.nu * m.nv, np = lay * m.nlayers;
    for (int64_t pt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pt < np;
         pt += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = pt / lay, r2 = pt - k * lay, j = r2 / m.nu, i = r2 - j * m.nu;
        double r0[3];
        point_pos(m, i, j, k, r0);
        const int64_t hb = pt, hf = m.nlines + pt;
        uint16_t st = m.rec.st[hb] | m.rec.st[hf];
        const int fb = m.rec.face[hb], ff = m.rec.face[hf];
        double eb[3], ef[3];
        for (int a = 0; a < 3; a++) {
            eb[a] = m.rec.end[3 * hb + a];
            ef[a] = m.rec.end[3 * hf + a];
        }
        if (edge_end(m, fb, eb) || edge_end(m, ff, ef)) st |= FQ_ST_EDGE;
        double q = NAN, qp = NAN, tw = NAN, len = NAN;
        if (!(st & kFatal)) {
            tw = m.rec.tw[hb] + m.rec.tw[hf];
            len = m.rec.len[hb] + m.rec.len[hf];
            const double *w1 = m.rec.uv + 6 * hb, *w2 = m.rec.uv + 6 * hf;
            const double U1[3] = {w1[0], w1[1], w1[2]}, V1[3] = {w1[3], w1[4], w1[5]};
            const double U2[3] = {w2[0], w2[1], w2[2]}, V2[3] = {w2[3], w2[4], w2[5]};
            double B0[3], B1[3], B2[3];
            field64(m, r0, B0);
            field64(m, eb, B1);
            field64(m, ef, B2);
            const double b00 = dot3(B0, B0);
            double n1[3] = {0, 0, 0}, n2[3] = {0, 0, 0}, u1[3], v1[3], u2[3], v2[3];
            n1[fb >> 1] = 1.0;
            n2[ff >> 1] = 1.0;
            along_b(U1, n1, B1, u1);
            along_b(V1, n1, B1, v1);
            along_b(U2, n2, B2, u2);
            along_b(V2, n2, B2, v2);
            q = scott(u1, v1, u2, v2) * fabs(comp3(B1, fb >> 1) * comp3(B2, ff >> 1)) / b00;
            const double m1 = sqrt(dot3(B1, B1)), m2 = sqrt(dot3(B2, B2));
            const double t1[3] = {B1[0] / m1, B1[1] / m1, B1[2] / m1};
            const double t2[3] = {B2[0] / m2, B2[1] / m2, B2[2] / m2};
            along_b(U1, t1, B1, u1);
            along_b(V1, t1, B1, v1);
            along_b(U2, t2, B2, u2);
            along_b(V2, t2, B2, v2);
            qp = scott(u1, v1, u2, v2) * m1 * m2 / b00;
        }
        if (m.out.q) m.out.q[pt] = q;
        if (m.out.qperp) m.out.qperp[pt] = qp;
        if (m.out.tw) m.out.tw[pt] = tw;
        if (m.out.length) m.out.length[pt] = len;
        if (m.out.status) m.out.status[pt] = st;
        const fq_lines &o = m.out.lines;
        if (o.end_b || o.end_f || o.face_b || o.face_f || o.bn_b || o.bn_f || o.bn0 || o.tw ||
            o.length || o.status)
            write_line(m, o, pt, r0);
    }
}

// Method I with S1, S2 perpendicular to B at the ends (Q_perp, Section 2.1), and the
// length edge map |grad_S0 length|, on one layer of a map: the 3-D end displacements
// of the point's stencil (the neighbour rule of Q: central where both neighbours end
// on the centre line's faces, else one-sided), projected along B onto the planes
// perpendicular to B at the ends. With P1, P2 the projected 3 x 2 Jacobians and
// G = P^T P, the map between the perpendicular sections has squared norm
// tr(G1^-1 G2) and determinant |B1 / B2|; det G1 = (Bn0 / |B1|)^2 from the flux
// through S0 (as Eq. D+-3 does for Q), so Q_perp = tr(adj(G1) G2) |B1| |B2| / Bn0^2.
// Points whose S0 is rotated get NaN. want_qperp = 0: the length edge map only
// (Method II forms its own Q_perp).

// One S0 axis: the S1 and S2 end displacements and the length change per unit seed
// coordinate, from the usable neighbours at pt - stride (if hm) and pt + stride (if
// hp). False when neither is usable.
__device__ __forceinline__ bool axis_diff3(const MapJob &m, const Line &c, int64_t pt, int64_t stride,
                                           bool hm, bool hp, double delta, double j1[3], double j2[3],
                                           double &dl)
{
    Line lm, lp;
    bool okm = false, okp = false;
    if (hm) {
        read_line(m.rec, m.nlines, pt - stride, lm);
        okm = !(lm.st & kFatal) && lm.f1 == c.f1 && lm.f2 == c.f2;
    }
    if (hp) {
        read_line(m.rec, m.nlines, pt + stride, lp);
        okp = !(lp.st & kFatal) && lp.f1 == c.f1 && lp.f2 == c.f2;
    }
    if (!okm && !okp) return false;
    const Line &lo = okm ? lm : c, &hi = okp ? lp : c;
    const double inv = 1.0 / ((okm && okp) ? 2.0 * delta : delta);
    for (int a = 0; a < 3; a++) {
        j1[a] = (hi.e1[a] - lo.e1[a]) * inv;
        j2[a] = (hi.e2[a] - lo.e2[a]) * inv;
    }
    dl = (hi.len - lo.len) * inv;
    return true;
}

// v minus its component along the unit vector t
__device__ __forceinline__ void perp3(double v[3], const double t[3])
{
    const double d = v[0] * t[0] + v[1] * t[1] + v[2] * t[2];
    for (int a = 0; a < 3; a++) v[a] -= d * t[a];
}

__global__ __launch_bounds__(256) void perp_kernel(MapJob m, int want_qperp)
{
    const int64_t lay = m.nu * m.nv, np = lay * m.nlayers;
    for (int64_t pt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pt < np;
         pt += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = pt / lay, r2 = pt - k * lay, j = r2 / m.nu, i = r2 - j * m.nu;
        Line c;
        read_line(m.rec, m.nlines, pt, c);
        double qp = NAN, fl = NAN;
        const int32_t ri = m.rot_index ? m.rot_index[pt] : -1;
        double jx1[3], jx2[3], jy1[3], jy2[3], dlx, dly;
        if (!(c.st & kFatal) && ri == -1 &&
            axis_diff3(m, c, pt, 1, i > 0, i < m.nu - 1, m.d0, jx1, jx2, dlx) &&
            axis_diff3(m, c, pt, m.nu, j > 0, j < m.nv - 1, m.d1, jy1, jy2, dly)) {
            fl = sqrt(dlx * dlx + dly * dly);
            if (want_qperp) {
                double r0[3], B0[3], B1[3], B2[3];
                point_pos(m, i, j, k, r0);
                field64(m, r0, B0);
                field64(m, c.e1, B1);
                field64(m, c.e2, B2);
                const double bn0 = B0[0] * m.normal[0] + B0[1] * m.normal[1] + B0[2] * m.normal[2];
                const double m1 = sqrt(dot3(B1, B1)), m2 = sqrt(dot3(B2, B2));
                const double t1[3] = {B1[0] / m1, B1[1] / m1, B1[2] / m1};
                const double t2[3] = {B2[0] / m2, B2[1] / m2, B2[2] / m2};
                perp3(jx1, t1);
                perp3(jy1, t1);
                perp3(jx2, t2);
                perp3(jy2, t2);
                const double g11 = dot3(jx1, jx1), g12 = dot3(jx1, jy1), g22 = dot3(jy1, jy1);
                const double h11 = dot3(jx2, jx2), h12 = dot3(jx2, jy2), h22 = dot3(jy2, jy2);
                qp = (g22 * h11 - 2.0 * g12 * h12 + g11 * h22) * m1 * m2 / (bn0 * bn0);
            }
        }
        if (want_qperp && m.out.qperp) m.out.qperp[pt] = qp;
        if (m.out.fledge) m.out.fledge[pt] = fl;
    }
}

// Method I on a cylindrical mapping surface (Section 3's x^2 + y^2 = 1 example): the
// point's stencil along theta and z, end coordinates (R theta, z) on the cylinder
// (arc lengths taken on the centre line's branch) or in-face ones on a box face,
// and Eq. D+-2, D+-3, Q+- with normal fields along the cylinder's outward normal.
__device__ __forceinline__ void cyl_uv(const MapJob &m, int face, const double e[3], double uv[2])
{
    if (face == kFaceCyl) {
        uv[0] = m.cyl[2] * atan2(e[1] - m.cyl[1], e[0] - m.cyl[0]);
        uv[1] = e[2];
    } else {
        inface(face, e, uv);
    }
}

__device__ __forceinline__ double unwrap(const MapJob &m, double u, double ref)
{
    const double turn = 2.0 * M_PI * m.cyl[2];
    return u - turn * rint((u - ref) / turn);
}

// One stencil axis: derivatives of the S1 and S2 end coordinates per unit seed
// coordinate from the usable neighbours at pt -+ stride (central, else one-sided).
__device__ __forceinline__ bool cyl_axis(const MapJob &m, const Line &c, int64_t pt, int64_t stride,
                                         bool hm, bool hp, double delta, double d1[2], double d2[2],
                                         uint16_t &st)
{
    Line lm, lp;
    bool okm = false, okp = false;
    if (hm) {
        read_line(m.rec, m.nlines, pt - stride, lm);
        okm = !(lm.st & kFatal) && lm.f1 == c.f1 && lm.f2 == c.f2;
        if (edge_end(m, lm.f1, lm.e1) || edge_end(m, lm.f2, lm.e2)) st |= FQ_ST_EDGE;
    }
    if (hp) {
        read_line(m.rec, m.nlines, pt + stride, lp);
        okp = !(lp.st & kFatal) && lp.f1 == c.f1 && lp.f2 == c.f2;
        if (edge_end(m, lp.f1, lp.e1) || edge_end(m, lp.f2, lp.e2)) st |= FQ_ST_EDGE;
    }
    if (!okm && !okp) return false;
    if (!(okm && okp)) st |= FQ_ST_ONESIDED;
    const Line &lo = okm ? lm : c, &hi = okp ? lp : c;
    double c1[2], c2[2], l1[2], l2[2], h1[2], h2[2];
    cyl_uv(m, c.f1, c.e1, c1);
    cyl_uv(m, c.f2, c.e2, c2);
    cyl_uv(m, lo.f1, lo.e1, l1);
    cyl_uv(m, lo.f2, lo.e2, l2);
    cyl_uv(m, hi.f1, hi.e1, h1);
    cyl_uv(m, hi.f2, hi.e2, h2);
    if (c.f1 == kFaceCyl) l1[0] = unwrap(m, l1[0], c1[0]), h1[0] = unwrap(m, h1[0], c1[0]);
    if (c.f2 == kFaceCyl) l2[0] = unwrap(m, l2[0], c2[0]), h2[0] = unwrap(m, h2[0], c2[0]);
    const double inv = 1.0 / ((okm && okp) ? 2.0 * delta : delta);
    for (int q = 0; q < 2; q++) {
        d1[q] = (h1[q] - l1[q]) * inv;
        d2[q] = (h2[q] - l2[q]) * inv;
    }
    return true;
}

__global__ __launch_bounds__(256) void cyl_map_kernel(MapJob m)
{
    const int64_t np = m.nu * m.nv;
    for (int64_t pt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pt < np;
         pt += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = pt / m.nu, i = pt - j * m.nu;
        const double t = m.p_origin[0] + (double)i * m.p_a[0];
        const double r0[3] = {m.cyl[0] + m.cyl[2] * cos(t), m.cyl[1] + m.cyl[2] * sin(t),
                              m.p_origin[1] + (double)j * m.p_b[1]};
        Line c;
        read_line(m.rec, m.nlines, pt, c);
        uint16_t st = c.st;
        if (edge_end(m, c.f1, c.e1) || edge_end(m, c.f2, c.e2)) st |= FQ_ST_EDGE;
        double q = NAN, tw = NAN, len = NAN;
        if (!(c.st & kFatal)) {
            tw = c.tw;
            len = c.len;
            double d1x[2], d2x[2], d1y[2], d2y[2];
            if (cyl_axis(m, c, pt, 1, i > 0, i < m.nu - 1, m.d0, d1x, d2x, st) &&
                cyl_axis(m, c, pt, m.nu, j > 0, j < m.nv - 1, m.d1, d1y, d2y, st)) {
                double B0[3], B1[3], B2[3];
                field64(m, r0, B0);
                field64(m, c.e1, B1);
                field64(m, c.e2, B2);
                const double bn0 = end_bn(m, kFaceCyl, r0, B0);
                const double bn1 = end_bn(m, c.f1, c.e1, B1), bn2 = end_bn(m, c.f2, c.e2, B2);
                // Eq. D+-3: (D10)^-1 = adj(D10) / |Bn0/Bn1|; Eq. D+-2: D12 = D20 (D10)^-1
                const double s = fabs(bn0 / bn1);
                const double i00 = d1y[1] / s, i01 = -d1y[0] / s, i10 = -d1x[1] / s, i11 = d1x[0] / s;
                const double a = d2x[0] * i00 + d2y[0] * i10, b = d2x[0] * i01 + d2y[0] * i11;
                const double cc = d2x[1] * i00 + d2y[1] * i10, d = d2x[1] * i01 + d2y[1] * i11;
                q = (a * a + b * b + cc * cc + d * d) / fabs(bn1 / bn2);
            } else {
                st |= FQ_ST_MIXEDFACE;
            }
        }
        if (m.out.q) m.out.q[pt] = q;
        if (m.out.tw) m.out.tw[pt] = tw;
        if (m.out.length) m.out.length[pt] = len;
        if (m.out.status) m.out.status[pt] = st;
        const fq_lines &o = m.out.lines;
        if (o.end_b || o.end_f || o.face_b || o.face_f || o.bn_b || o.bn_f || o.bn0 || o.tw ||
            o.length || o.status)
            write_line(m, o, pt, r0);
    }
}

__global__ void lines_kernel(MapJob m, const double *seeds)
{
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < m.nlines;
         l += (int64_t)gridDim.x * blockDim.x) {
        const double s[3] = {seeds[3 * l], seeds[3 * l + 1], seeds[3 * l + 2]};
        write_line(m, m.out.lines, l, s);
    }
}

unsigned blocks_for(int64_t n)
{
    int64_t b = (n + 255) / 256;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return (unsigned)b;
}

}  // namespace

hipError_t launch_classify(const MapJob &m, int32_t *rot_index, RotEntry *rot,
                           uint32_t *rot_count, int64_t capacity, hipStream_t s)
{
    const int64_t np = m.nu * m.nv * m.nlayers;
    hipLaunchKernelGGL(classify_kernel, dim3(blocks_for(np)), dim3(256), 0, s, m, rot_index, rot,
                       rot_count, capacity);
    return hipGetLastError();
}

hipError_t launch_stencil(const MapJob &m, hipStream_t s)
{
    const int64_t np = m.nu * m.nv * m.nlayers;
    hipLaunchKernelGGL(stencil_kernel, dim3(blocks_for(np)), dim3(256), 0, s, m);
    return hipGetLastError();
}

hipError_t launch_m2_map(const MapJob &m, hipStream_t s)
{
    const int64_t np = m.nu * m.nv * m.nlayers;
    hipLaunchKernelGGL(m2_map_kernel, dim3(blocks_for(np)), dim3(256), 0, s, m);
    return hipGetLastError();
}

hipError_t launch_perp_map(const MapJob &m, int want_qperp, hipStream_t s)
{
    const int64_t np = m.nu * m.nv * m.nlayers;
    hipLaunchKernelGGL(perp_kernel, dim3(blocks_for(np)), dim3(256), 0, s, m, want_qperp);
    return hipGetLastError();
}

hipError_t launch_cyl_map(const MapJob &m, hipStream_t s)
{
    hipLaunchKernelGGL(cyl_map_kernel, dim3(blocks_for(m.nu * m.nv)), dim3(256), 0, s, m);
    return hipGetLastError();
}

hipError_t launch_lines_out(const MapJob &m, const double *seeds, hipStream_t s)
{
    hipLaunchKernelGGL(lines_kernel, dim3(blocks_for(m.nlines)), dim3(256), 0, s, m, seeds);
    return hipGetLastError();
}

}  // namespace fq
