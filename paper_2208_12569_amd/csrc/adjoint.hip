// Reverse-mode derivative of a Q/Tw map with respect to the field's node values.
//
// The map is a composition: node values -> (curl by differences) -> cell
// polynomials -> traced half lines (ends, Tw) -> Method-I stencil (Q, Section 2.1
// Eq. D+-2 / D+-3, Section 1 Eq. Q+-) with the normal fields Bn0, Bn1, Bn2
// interpolated from the nodes. Its adjoint runs the other way:
//   map_backward   dL/dQ, dL/dTw, dL/d(ends) -> dL/d(end of every half line),
//                  dL/d(Tw of every half line), and dL/dB at the nodes through
//                  the trilinear Bn0, Bn1, Bn2;
//   trace_backward the discrete adjoint of every accepted Runge-Kutta step of a half
//                  line, last to first, with the step lengths held fixed: the
//                  forward pass kept the lane state every `seg` accepted steps
//                  (chained per half line in one checkpoint pool),
//                  and each segment is replayed from its checkpoint with the same
//                  stepping code (bit-identical), its accepted steps recorded, and
//                  then swept in reverse; gradients with respect to the 8 corner
//                  values of B and curl B of each cell go to the nodes;
//   grad_planes    adds dL/dB of the nodes and the transpose of the curl
//                  differences applied to dL/d(curl B) into the caller's planes.
// All of it is FP64.
#include <math.h>

#include "fq_internal.h"
#include "stencil_dev.h"
#include "trace_core.h"
#include "trace_dev.h"

namespace fq {
namespace {

using namespace dev;
using namespace sten;

// ----------------------------------------------------------------------------------
// Trilinear weights of the caller's planes at a physical point (the cell choice of
// the FP64 interpolation), and their derivatives along x, y, z.
struct Tri {
    int64_t node[8];
    double w[8];
    double dw[8][3];
};

__device__ void tri_of(const MapJob &m, const double r[3], Tri &t)
{
    int c[3];
    double u[3], iw[3];
    for (int a = 0; a < 3; a++) {
        if (m.coord[a]) {
            // a stretched axis: the cell by bisection, as the FP64 interpolation
            const double *x = m.coord[a];
            const int ci = axis_cell(x, m.n[a], r[a]);
            c[a] = ci;
            iw[a] = 1.0 / (x[ci + 1] - x[ci]);
            u[a] = (r[a] - x[ci]) * iw[a];
            continue;
        }
        const double g = (r[a] - m.origin[a]) / m.spacing[a];
        int ci = (int)floor(g);
        ci = ci < 0 ? 0 : (ci > m.n[a] - 2 ? m.n[a] - 2 : ci);
        c[a] = ci;
        u[a] = g - ci;
        iw[a] = 1.0 / m.spacing[a];
    }
    const int64_t sy = m.n[0], sz = (int64_t)m.n[0] * m.n[1];
    const int64_t base = c[2] * sz + c[1] * sy + c[0];
    for (int q = 0; q < 8; q++) {
        const int ix = q & 1, iy = (q >> 1) & 1, iz = (q >> 2) & 1;
        const double wx = ix ? u[0] : 1.0 - u[0], wy = iy ? u[1] : 1.0 - u[1],
                     wz = iz ? u[2] : 1.0 - u[2];
        const double sx = ix ? 1.0 : -1.0, syy = iy ? 1.0 : -1.0, szz = iz ? 1.0 : -1.0;
        t.node[q] = base + ix + iy * sy + iz * sz;
        t.w[q] = wx * wy * wz;
        t.dw[q][0] = sx * wy * wz * iw[0];
        t.dw[q][1] = wx * syy * wz * iw[1];
        t.dw[q][2] = wx * wy * szz * iw[2];
    }
}

__device__ __forceinline__ double plane_at(const MapJob &m, int comp, int64_t o)
{
    return m.dtype == FQ_DT_F32 ? (double)((const float *)m.b[comp])[o]
                                : ((const double *)m.b[comp])[o];
}

// d B_comp / d r at the point of t
__device__ void grad_comp(const MapJob &m, const Tri &t, int comp, double g[3])
{
    g[0] = g[1] = g[2] = 0.0;
    for (int q = 0; q < 8; q++) {
        const double v = plane_at(m, comp, t.node[q]);
        g[0] += t.dw[q][0] * v;
        g[1] += t.dw[q][1] * v;
        g[2] += t.dw[q][2] * v;
    }
}

// adjoint of the two in-face coordinates of an end (face f) -> end point adjoint
__device__ __forceinline__ void inface_adj(int face, const double ub[2], double eb[3])
{
    // by selects: an index computed at run time would put eb in scratch memory
    const int a = face >> 1;
    if (a == 0) eb[1] += ub[0];
    else eb[0] += ub[0];
    if (a == 2) eb[1] += ub[1];
    else eb[2] += ub[1];
}

__device__ __forceinline__ void add3(double *dst, const double v[3])
{
    for (int a = 0; a < 3; a++)
        if (v[a] != 0.0) atomicAdd(dst + a, v[a]);
}

// End adjoints of one line of the stencil, kept in S1 / S2 order.
struct LineAdj {
    double e1[3], e2[3];
};

// Adjoint of the derivatives along one S0 axis (d1 of (u1,v1), d2 of (u2,v2)) onto
// the in-face coordinates of the lines the difference used.
__device__ __forceinline__ void axis_adj(int rule, const Line &c, const Nb &m, const Nb &p, double d,
                         const double d1b[2], const double d2b[2], LineAdj &cb, LineAdj &mb,
                         LineAdj &pb)
{
    double s_p = 0.0, s_m = 0.0, s_c = 0.0;
    if (rule == RULE_CENTRAL) s_p = 0.5 / d, s_m = -0.5 / d;
    else if (rule == RULE_PLUS) s_p = 1.0 / d, s_c = -1.0 / d;
    else s_c = 1.0 / d, s_m = -1.0 / d;
    double u1[2], u2[2];
    if (s_p != 0.0) {
        u1[0] = s_p * d1b[0], u1[1] = s_p * d1b[1];
        u2[0] = s_p * d2b[0], u2[1] = s_p * d2b[1];
        inface_adj(p.f1, u1, pb.e1);
        inface_adj(p.f2, u2, pb.e2);
    }
    if (s_m != 0.0) {
        u1[0] = s_m * d1b[0], u1[1] = s_m * d1b[1];
        u2[0] = s_m * d2b[0], u2[1] = s_m * d2b[1];
        inface_adj(m.f1, u1, mb.e1);
        inface_adj(m.f2, u2, mb.e2);
    }
    if (s_c != 0.0) {
        u1[0] = s_c * d1b[0], u1[1] = s_c * d1b[1];
        u2[0] = s_c * d2b[0], u2[1] = s_c * d2b[1];
        inface_adj(c.f1, u1, cb.e1);
        inface_adj(c.f2, u2, cb.e2);
    }
}

// S1 / S2 end adjoints of line l (of a job of nlines lines) -> the half records
__device__ __forceinline__ void push_line_n(int64_t nlines, int64_t l, bool swapped, const LineAdj &a,
                                            double *lam_end)
{
    const int64_t hb = l, hf = nlines + l;
    const int64_t s1 = swapped ? hf : hb, s2 = swapped ? hb : hf;
    add3(lam_end + 3 * s1, a.e1);
    add3(lam_end + 3 * s2, a.e2);
}

__device__ __forceinline__ void push_line(const MapJob &m, int64_t l, bool swapped, const LineAdj &a,
                                          double *lam_end)
{
    const int64_t hb = l, hf = m.nlines + l;
    const int64_t s1 = swapped ? hf : hb, s2 = swapped ? hb : hf;
    add3(lam_end + 3 * s1, a.e1);
    add3(lam_end + 3 * s2, a.e2);
}

__device__ void bn_adj(const MapJob &m, const double r[3], int comp, double gbn, double eb[3],
                       double *gnode, int64_t nn)
{
    Tri t;
    tri_of(m, r, t);
    if (eb) {
        double g[3];
        grad_comp(m, t, comp, g);
        for (int a = 0; a < 3; a++) eb[a] += gbn * g[a];
    }
    for (int q = 0; q < 8; q++) atomicAdd(gnode + comp * nn + t.node[q], gbn * t.w[q]);
}

__global__ __launch_bounds__(256) void map_backward_kernel(MapJob m, const double *__restrict__ dq,
                                    const double *__restrict__ dtw,
                                    const double *__restrict__ dend_b,
                                    const double *__restrict__ dend_f, double *lam_end,
                                    double *lam_tw, double *gnode, int64_t nhalf0)
{
    // a 3-D map's layers each take the plane's stencil, with neighbours in the layer
    const int64_t lay = m.nu * m.nv, np = lay * m.nlayers;
    const int64_t nn = (int64_t)m.n[0] * m.n[1] * m.n[2];
    for (int64_t pt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pt < np;
         pt += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = pt / lay, r2 = pt - k * lay, j = r2 / m.nu, i = r2 - j * m.nu;
        Line c;
        read_line(m.rec, m.nlines, pt, c);
        if (c.st & kFatal) continue;
        const int64_t hb = pt, hf = m.nlines + pt;
        // Tw of the point is the sum of its two halves
        if (dtw && isfinite(dtw[pt])) {
            lam_tw[hb] = dtw[pt];
            lam_tw[hf] = dtw[pt];
        }
        if (dend_b) {
            const double v[3] = {dend_b[3 * pt], dend_b[3 * pt + 1], dend_b[3 * pt + 2]};
            if (isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2])) add3(lam_end + 3 * hb, v);
        }
        if (dend_f) {
            const double v[3] = {dend_f[3 * pt], dend_f[3 * pt + 1], dend_f[3 * pt + 2]};
            if (isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2])) add3(lam_end + 3 * hf, v);
        }
        if (!dq) continue;
        const double gq = dq[pt];
        if (!(gq != 0.0) || !isfinite(gq)) continue;
        // a rotated S0 (Section 4): the four lines seeded at r0 -+ delta U, r0 -+ delta V
        // of the rotated-S0 job stand in for the neighbours, central differences over
        // delta, and |B0| for Bn0
        const int32_t ri = m.rot_index ? m.rot_index[pt] : -1;
        if (ri == -2) continue;  // no Q there
        const bool rot = ri >= 0;
        const int64_t r4 = 4 * (int64_t)(rot ? ri : 0);
        const bool hxm = rot || i > 0, hxp = rot || i < m.nu - 1, hym = rot || j > 0,
                   hyp = rot || j < m.nv - 1;
        // a missing neighbour reads the centre's own record (never used)
        const Nb xm = rot ? read_nb(m, m.rot_rec, m.rot_nlines, r4 + 0) : read_nb(m, m.rec, m.nlines, hxm ? pt - 1 : pt);
        const Nb xp = rot ? read_nb(m, m.rot_rec, m.rot_nlines, r4 + 1) : read_nb(m, m.rec, m.nlines, hxp ? pt + 1 : pt);
        const Nb ym = rot ? read_nb(m, m.rot_rec, m.rot_nlines, r4 + 2) : read_nb(m, m.rec, m.nlines, hym ? pt - m.nu : pt);
        const Nb yp = rot ? read_nb(m, m.rot_rec, m.rot_nlines, r4 + 3) : read_nb(m, m.rec, m.nlines, hyp ? pt + m.nu : pt);
        const double dx = rot ? m.rot_delta : m.d0, dy = rot ? m.rot_delta : m.d1;
        const int rx = axis_rule(c, xm, hxm, xp, hxp), ry = axis_rule(c, ym, hym, yp, hyp);
        if (rx == RULE_NONE || ry == RULE_NONE) continue;  // Q = NaN there
        uint16_t st = 0;
        double c1[2], c2[2];
        inface(c.f1, c.e1, c1);
        inface(c.f2, c.e2, c2);
        double ax1[2], ax2[2], ay1[2], ay2[2];
        axis_diff(rx, c1, c2, xm, xp, dx, ax1, ax2, st);
        axis_diff(ry, c1, c2, ym, yp, dy, ay1, ay2, st);
        const double j00 = ax1[0], j01 = ay1[0], j10 = ax1[1], j11 = ay1[1];
        const double k00 = ax2[0], k01 = ay2[0], k10 = ax2[1], k11 = ay2[1];
        const double m00 = k00 * j11 - k01 * j10;
        const double m01 = -k00 * j01 + k01 * j00;
        const double m10 = k10 * j11 - k11 * j10;
        const double m11 = -k10 * j01 + k11 * j00;
        double r0[3], B0[3], B1[3], B2[3];
        point_pos(m, i, j, k, r0);
        field64(m, r0, B0);
        field64(m, c.e1, B1);
        field64(m, c.e2, B2);
        const double bn0 = rot ? sqrt(B0[0] * B0[0] + B0[1] * B0[1] + B0[2] * B0[2])
                               : B0[0] * m.normal[0] + B0[1] * m.normal[1] + B0[2] * m.normal[2];
        const int a1 = c.f1 >> 1, a2 = c.f2 >> 1;
        const double bn1 = comp3(B1, a1), bn2 = comp3(B2, a2);
        const double nrm = m00 * m00 + m01 * m01 + m10 * m10 + m11 * m11;
        const double A = fabs(bn1 * bn2) / (bn0 * bn0);
        const double Q = nrm * A;
        if (!isfinite(Q) || !(bn1 != 0.0) || !(bn2 != 0.0)) continue;
        // Q = ||M||^2 A, M = J2 adj(J1)
        const double s = 2.0 * gq * A;
        const double M00 = s * m00, M01 = s * m01, M10 = s * m10, M11 = s * m11;
        const double kb00 = M00 * j11 - M01 * j01, kb01 = -M00 * j10 + M01 * j00;
        const double kb10 = M10 * j11 - M11 * j01, kb11 = -M10 * j10 + M11 * j00;
        const double jb00 = M01 * k01 + M11 * k11, jb01 = -M01 * k00 - M11 * k10;
        const double jb10 = -M00 * k01 - M10 * k11, jb11 = M00 * k00 + M10 * k10;
        LineAdj ca = {}, xma = {}, xpa = {}, yma = {}, ypa = {};
        {
            const double d1b[2] = {jb00, jb10}, d2b[2] = {kb00, kb10};
            axis_adj(rx, c, xm, xp, dx, d1b, d2b, ca, xma, xpa);
        }
        {
            const double d1b[2] = {jb01, jb11}, d2b[2] = {kb01, kb11};
            axis_adj(ry, c, ym, yp, dy, d1b, d2b, ca, yma, ypa);
        }
        // the normal fields: Q ~ |Bn1 Bn2| / Bn0^2
        bn_adj(m, c.e1, a1, gq * Q / bn1, ca.e1, gnode, nn);
        bn_adj(m, c.e2, a2, gq * Q / bn2, ca.e2, gnode, nn);
        const double gb0 = -2.0 * gq * Q / bn0;
        // Bn0 = n.B0, or |B0| on a rotated S0 (d|B0| / dB0 = B0 / |B0|)
        for (int comp = 0; comp < 3; comp++) {
            const double w = rot ? B0[comp] / bn0 : m.normal[comp];
            if (w != 0.0) bn_adj(m, r0, comp, gb0 * w, nullptr, gnode, nn);
        }
        push_line(m, pt, c.swapped, ca, lam_end);
        if (rot) {
            // the rotated-S0 job's records follow the plane's in the adjoint arrays
            double *lr = lam_end + 3 * nhalf0;
            push_line_n(m.rot_nlines, r4 + 0, xm.swapped, xma, lr);
            push_line_n(m.rot_nlines, r4 + 1, xp.swapped, xpa, lr);
            push_line_n(m.rot_nlines, r4 + 2, ym.swapped, yma, lr);
            push_line_n(m.rot_nlines, r4 + 3, yp.swapped, ypa, lr);
        } else {
            if (rx != RULE_PLUS) push_line(m, pt - 1, xm.swapped, xma, lam_end);
            if (rx != RULE_MINUS) push_line(m, pt + 1, xp.swapped, xpa, lam_end);
            if (ry != RULE_PLUS) push_line(m, pt - m.nu, ym.swapped, yma, lam_end);
            if (ry != RULE_MINUS) push_line(m, pt + m.nu, yp.swapped, ypa, lam_end);
        }
    }
}

// ----------------------------------------------------------------------------------
// Discrete adjoint of one accepted Runge-Kutta step (FP64).

// value and gradient (local coordinates) of P(u,v,w) in monomial form
template <typename T>
__device__ __forceinline__ void poly_grad(const T c[8], T u, T v, T w, T g[3])
{
    g[0] = c[1] + c[4] * v + c[5] * w + c[7] * v * w;
    g[1] = c[2] + c[4] * u + c[6] * w + c[7] * u * w;
    g[2] = c[3] + c[5] * u + c[6] * v + c[7] * u * v;
}

template <typename T> __device__ __forceinline__ T tri_w(int q, T u, T v, T w)
{
    return ((q & 1) ? u : T(1) - u) * ((q & 2) ? v : T(1) - v) * ((q & 4) ? w : T(1) - w);
}

// The tableaux the forward step uses, by Scheme: Fehlberg 4(5) with its fifth-order
// weights; classic RK4; Kutta's 3/8 rule (the two RK4 rules use stages 0-3).
__constant__ double kA[3][6][5] = {
    {{0.0, 0.0, 0.0, 0.0, 0.0},
     {1.0 / 4.0, 0.0, 0.0, 0.0, 0.0},
     {3.0 / 32.0, 9.0 / 32.0, 0.0, 0.0, 0.0},
     {1932.0 / 2197.0, -7200.0 / 2197.0, 7296.0 / 2197.0, 0.0, 0.0},
     {439.0 / 216.0, -8.0, 3680.0 / 513.0, -845.0 / 4104.0, 0.0},
     {-8.0 / 27.0, 2.0, -3544.0 / 2565.0, 1859.0 / 4104.0, -11.0 / 40.0}},
    {{0.0, 0.0, 0.0, 0.0, 0.0},
     {0.5, 0.0, 0.0, 0.0, 0.0},
     {0.0, 0.5, 0.0, 0.0, 0.0},
     {0.0, 0.0, 1.0, 0.0, 0.0},
     {0.0, 0.0, 0.0, 0.0, 0.0},
     {0.0, 0.0, 0.0, 0.0, 0.0}},
    {{0.0, 0.0, 0.0, 0.0, 0.0},
     {1.0 / 3.0, 0.0, 0.0, 0.0, 0.0},
     {-1.0 / 3.0, 1.0, 0.0, 0.0, 0.0},
     {1.0, -1.0, 1.0, 0.0, 0.0},
     {0.0, 0.0, 0.0, 0.0, 0.0},
     {0.0, 0.0, 0.0, 0.0, 0.0}}};
__constant__ double kB[3][6] = {
    {16.0 / 135.0, 0.0, 6656.0 / 12825.0, 28561.0 / 56430.0, -9.0 / 50.0, 2.0 / 55.0},
    {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0, 0.0, 0.0},
    {1.0 / 8.0, 3.0 / 8.0, 3.0 / 8.0, 1.0 / 8.0, 0.0, 0.0}};

// The accepted step maps local position p to p' (a plain step of arc length H, or a
// landing with the axis coordinate as the independent variable, H = face - p_axis)
// and adds H * sum b_s G_s / g_s to Tw (G = twk (J.B)/|B|^2, g = 1 or dp_axis/ds).
// Given lam = dL/dp' and ltw = dL/dTw, returns lam = dL/dp and adds dL/d(corner
// values) of B and curl B to gB, gJ.
// endb: for the last accepted step of a half line, the axis of the box face the line
// ends on (-1 otherwise).
// T: the arithmetic of the sweep, FP64, or FP32 in the F32X form (whose forward
// steps were FP32); the callers accumulate gB, gJ per cell and add them to FP64
// node gradients.
template <typename T, bool TW, int SCH>
__device__ void step_adjoint(const T cb[3][8], const T cj[3][8], const StepRec &sr,
                             const LaneConst<T> &K, T sgn, int endb, T lam[3], T ltw, T gB[3][8],
                             T gJ[3][8])
{
    constexpr int NS = SCH == SCH_RKF45 ? 6 : 4;  // stages
    // the tableau, read where it is used (the loops are over uniform indices)
    auto A = [](int st, int jj) { return (T)kA[SCH][st][jj]; };
    auto Bw = [](int st) { return (T)kB[SCH][st]; };
    const T R[3] = {K.rx, K.ry, K.rz};
    const T p[3] = {(T)sr.p0, (T)sr.p1, (T)sr.p2};
    const T H = (T)sr.H;
    const int ax = sr.axis;
    T y[6][3], k[6][3], G[6], g[6];
    for (int st = 0; st < NS; st++) {
        for (int q = 0; q < 3; q++) {
            T acc = T(0);
            for (int jj = 0; jj < st; jj++) acc += A(st, jj) * k[jj][q];
            y[st][q] = p[q] + H * acc;
        }
        T B[3], J[3] = {T(0), T(0), T(0)};
        for (int c = 0; c < 3; c++) B[c] = poly<T>(cb[c], y[st][0], y[st][1], y[st][2]);
        if (TW)
            for (int c = 0; c < 3; c++) J[c] = poly<T>(cj[c], y[st][0], y[st][1], y[st][2]);
        const T b2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
        const T inv = T(1) / sqrt(b2);
        T F[3];
        for (int c = 0; c < 3; c++) F[c] = sgn * inv * B[c] * R[c];
        G[st] = TW ? K.twk * (J[0] * B[0] + J[1] * B[1] + J[2] * B[2]) * inv * inv : T(0);
        g[st] = ax >= 0 ? F[ax] : 1.0;
        for (int c = 0; c < 3; c++) k[st][c] = F[c] / g[st];
    }
    // Adjoint of the outputs that depend on the step. A landing coordinate ends
    // exactly on its face. When the step puts the line on the box face b it ends on
    // without landing on it (the last step of the line landed on another face or was
    // a plain step, with b exactly on the face or clamped onto it), that box face is
    // the end constraint: the landing (if any) is incidental, the step length is held
    // fixed, and the end moves along the line's direction onto the face,
    // p_end = p* - k (p*_b - face_b) / k_b, whose adjoint is taken here.
    T lo[3];
    int b = -1;
    if (endb >= 0 && endb != ax) b = endb;
    else if (endb < 0 && sr.clamp) b = (sr.clamp & 1) ? 0 : ((sr.clamp & 2) ? 1 : 2);
    const bool onbox = b >= 0;
    if (!onbox) {
        for (int q = 0; q < 3; q++) lo[q] = q == ax ? T(0) : lam[q];
    } else {
        T pe[3];
        for (int q = 0; q < 3; q++) {
            T dy = T(0);
            for (int st = 0; st < NS; st++) dy += Bw(st) * k[st][q];
            pe[q] = p[q] + H * dy;
        }
        // direction F and twist integrand G at the end: moving the end by dt along the
        // line moves p by F dt and Tw by G dt, with dt = -(p*_b - face_b) / F_b
        T Be[3], Je[3] = {T(0), T(0), T(0)};
        for (int c = 0; c < 3; c++) Be[c] = poly<T>(cb[c], pe[0], pe[1], pe[2]);
        if (TW)
            for (int c = 0; c < 3; c++) Je[c] = poly<T>(cj[c], pe[0], pe[1], pe[2]);
        const T be2 = Be[0] * Be[0] + Be[1] * Be[1] + Be[2] * Be[2];
        const T inve = T(1) / sqrt(be2);
        T Fe[3];
        for (int c = 0; c < 3; c++) Fe[c] = sgn * inve * Be[c] * R[c];
        T s_ = T(0);
        for (int q = 0; q < 3; q++)
            if (q != b) s_ += lam[q] * Fe[q];
        if (TW) s_ += ltw * K.twk * (Je[0] * Be[0] + Je[1] * Be[1] + Je[2] * Be[2]) * inve * inve;
        for (int q = 0; q < 3; q++) lo[q] = q == b ? -s_ / Fe[b] : lam[q];
    }
    T mu[6][3];
    T dH = T(0);
    for (int st = 0; st < NS; st++) {
        for (int q = 0; q < 3; q++) mu[st][q] = H * Bw(st) * lo[q];
        dH += Bw(st) * (k[st][0] * lo[0] + k[st][1] * lo[1] + k[st][2] * lo[2]);
        if (TW) dH += ltw * Bw(st) * G[st] / g[st];
    }
    T ln[3] = {lo[0], lo[1], lo[2]};
    for (int st = NS - 1; st >= 0; st--) {
        const T u = y[st][0], v = y[st][1], w = y[st][2];
        T B[3], J[3] = {T(0), T(0), T(0)};
        for (int c = 0; c < 3; c++) B[c] = poly<T>(cb[c], u, v, w);
        if (TW)
            for (int c = 0; c < 3; c++) J[c] = poly<T>(cj[c], u, v, w);
        const T b2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
        const T inv = T(1) / sqrt(b2);
        const T tau = TW ? H * Bw(st) * ltw : T(0);
        T Fb[3], Gb;
        if (ax >= 0) {
            const T ig = 1.0 / g[st];
            const T mk = mu[st][0] * k[st][0] + mu[st][1] * k[st][1] + mu[st][2] * k[st][2];
            for (int c = 0; c < 3; c++) Fb[c] = mu[st][c] * ig;
            Gb = tau * ig;
            Fb[ax] += -mk * ig - tau * G[st] * ig * ig;
        } else {
            for (int c = 0; c < 3; c++) Fb[c] = mu[st][c];
            Gb = tau;
        }
        // F = sgn R (B / |B|)
        T d[3], db[3];
        for (int c = 0; c < 3; c++) {
            d[c] = B[c] * inv;
            db[c] = sgn * R[c] * Fb[c];
        }
        const T dd = db[0] * d[0] + db[1] * d[1] + db[2] * d[2];
        T Bb[3], Jb[3] = {T(0), T(0), T(0)};
        for (int c = 0; c < 3; c++) Bb[c] = (db[c] - dd * d[c]) * inv;
        if (TW && Gb != T(0)) {
            // G = twk (J.B) / |B|^2
            const T i2 = inv * inv;
            const T jb = J[0] * B[0] + J[1] * B[1] + J[2] * B[2];
            for (int c = 0; c < 3; c++) {
                Jb[c] = K.twk * Gb * B[c] * i2;
                Bb[c] += K.twk * Gb * (J[c] * i2 - T(2) * jb * i2 * i2 * B[c]);
            }
        }
        T yb[3] = {T(0), T(0), T(0)};
        for (int c = 0; c < 3; c++) {
            T gr[3];
            poly_grad(cb[c], u, v, w, gr);
            for (int a = 0; a < 3; a++) yb[a] += Bb[c] * gr[a];
            if (TW) {
                poly_grad(cj[c], u, v, w, gr);
                for (int a = 0; a < 3; a++) yb[a] += Jb[c] * gr[a];
            }
        }
        for (int q = 0; q < 8; q++) {
            const T wq = tri_w(q, u, v, w);
            for (int c = 0; c < 3; c++) {
                gB[c][q] += Bb[c] * wq;
                if (TW) gJ[c][q] += Jb[c] * wq;
            }
        }
        for (int a = 0; a < 3; a++) ln[a] += yb[a];
        for (int jj = 0; jj < st; jj++) {
            for (int a = 0; a < 3; a++) mu[jj][a] += H * A(st, jj) * yb[a];
            dH += A(st, jj) * (yb[0] * k[jj][0] + yb[1] * k[jj][1] + yb[2] * k[jj][2]);
        }
    }
    if (ax >= 0 && !onbox) ln[ax] -= dH;  // H = face - p_axis
    for (int a = 0; a < 3; a++) lam[a] = ln[a];
}

// Captures the accepted step of a replayed trial.
struct Capture {
    int *axis;
    double *H;
    int *clamp;
    __device__ __forceinline__ void operator()(int) const {}
    template <typename T> __device__ __forceinline__ void accepted(int a, T h, int cl) const
    {
        *axis = a;
        *H = (double)h;
        *clamp = cl;
    }
};

template <typename T, bool TW>
__device__ void flush_cell(double *gnode, int64_t nn, int nx, int ny, int c0, int c1, int c2,
                           T gB[3][8], T gJ[3][8])
{
    const int64_t sy = nx, sz = (int64_t)nx * ny;
    const int64_t base = (int64_t)c2 * sz + (int64_t)c1 * sy + c0;
    for (int q = 0; q < 8; q++) {
        const int64_t o = base + (q & 1) + ((q >> 1) & 1) * sy + ((q >> 2) & 1) * sz;
        for (int c = 0; c < 3; c++) {
            if (gB[c][q] != T(0)) atomicAdd(gnode + c * nn + o, (double)gB[c][q]);
            gB[c][q] = T(0);
            if (TW) {
                if (gJ[c][q] != T(0)) atomicAdd(gnode + (3 + c) * nn + o, (double)gJ[c][q]);
                gJ[c][q] = T(0);
            }
        }
    }
}

// T: the arithmetic of the replay (that of the forward pass, so the replay is bit
// for bit) and of the reverse sweep; S: the node records.
template <typename T, typename S, bool TW, int SCH>
__global__ __launch_bounds__(64) void trace_backward_kernel(const TraceJob *__restrict__ jobs,
                                                            BwdParams bp)
{
    const TraceJob &J = jobs[0];
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= bp.nslots) return;
    StepRec *buf = bp.buf + slot * bp.seg;
    LaneConst<T> K;
    K.nx = J.n[0];
    K.ny = J.n[1];
    K.nz = J.n[2];
    K.rx = (T)J.rscale[0];
    K.ry = (T)J.rscale[1];
    K.rz = (T)J.rscale[2];
    K.twk = (T)J.twk;
    K.bnull2 = (T)((double)Num<T>::null_rel * (double)(*J.bmax2));
    K.max_steps = bp.max_steps;
    // stretched grids: lengths in units of the smallest cell width, and every cell's
    // own scales (set with each cell, as the forward pass did)
    const bool str = J.geo != nullptr;
    const double dref = str ? J.geo->dref : 0.0;
    if (str) K.twk = (T)(dref * (0.25 / M_PI));
    auto cell_scales = [&](int c0, int c1, int c2) {
        if (!str) return;
        K.rx = (T)(dref * J.iw[0][c0]);
        K.ry = (T)(dref * J.iw[1][c1]);
        K.rz = (T)(dref * J.iw[2][c2]);
    };
    const int64_t nn = (int64_t)K.nx * K.ny * K.nz;
    unsigned long long n_half = 0, n_steps = 0, n_bad = 0, n_drop = 0;
    T cb[3][8], cj[3][8], gB[3][8], gJ[3][8];
    for (int c = 0; c < 3; c++)
        for (int q = 0; q < 8; q++) gB[c][q] = gJ[c][q] = T(0);
    // A lane reverses its half line one segment per iteration and takes the next half
    // line as soon as its own is done, so the lanes of a wave stay busy while their
    // half lines differ in length (a segment costs about the same everywhere).
    int64_t h = -1;       // the lane's half line, -1 = none
    bool drained = false; // the queue is empty
    T lam[3] = {T(0), T(0), T(0)}, ltw = T(0), sgn = T(1);
    int endax = -1, ckslot = -1, next = -1, ck = -1, nck = 0, nacc = 0, rj = 0;
    bool bad = false;
    for (;;) {
        while (h < 0 && !drained) {
            const unsigned long long hq = atomicAdd(bp.counter, 1ull);
            if (hq >= (unsigned long long)bp.nhalves) {
                drained = true;
                break;
            }
            // long half lines first: they set the end of the launch
            const int64_t hh = bp.order ? (int64_t)bp.order[hq] : (int64_t)hq;
            // the half's own job (a rotated-S0 job's halves follow the plane's) and
            // its record there
            rj = hh >= bp.nhalf0 ? 1 : 0;
            const TraceJob &Jh = jobs[rj];
            const int64_t lh = hh - (rj ? bp.nhalf0 : 0);
            // in physical units here; in local units (times the end cell's widths) once
            // the replay of the last segment has found that cell
            for (int a = 0; a < 3; a++) lam[a] = (T)bp.lam_end[3 * hh + a];
            // the end lies on its box face: only its in-face coordinates can move
            const int fe = Jh.rec.face[lh];
            if (fe >= 0) lam[fe >> 1] = T(0);
            endax = fe >= 0 ? (fe >> 1) : -1;
            ltw = TW ? (T)bp.lam_tw[hh] : T(0);
            if (lam[0] == T(0) && lam[1] == T(0) && lam[2] == T(0) && ltw == T(0)) continue;
            const uint16_t st = Jh.rec.st[lh];
            nck = bp.tape_n[hh];
            nacc = bp.tape_acc[hh];
            if (st & kFatal) {
                n_drop++;  // a line the forward map has but this pass could not keep
                continue;
            }
            if (nck <= 0 || nacc <= 0) continue;  // no step taken (a seed on its exit face)
            sgn = lh >= Jh.nlines ? T(1) : T(-1);
            n_half++;
            bad = false;
            ckslot = bp.tape_last[hh];
            next = -1;
            ck = nck - 1;
            h = hh;
        }
        if (__ballot(h >= 0) == 0) break;  // every lane is drained
        if (h < 0) continue;
        {
            // replay the segment from its checkpoint
            const Ckpt cp = bp.tape[ckslot];
            Lane<T> L;
            L.c0 = cp.c0, L.c1 = cp.c1, L.c2 = cp.c2;
            L.p0 = (T)cp.p0, L.p1 = (T)cp.p1, L.p2 = (T)cp.p2;
            L.h = (T)cp.h, L.tol = (T)cp.tol, L.sgn = sgn;
            L.tw = 0.0, L.len = 0.0;
            L.trials = cp.trials;
            L.force = cp.force;
            const bool last = ck == nck - 1;
            const int target = last ? nacc - ck * bp.seg : bp.seg;
            if (target < 0 || target > bp.seg || (target == 0 && !last)) bad = true;
            int nrec = 0;
            if (!bad) {
                load_cell<T, S, TW>(J.nodes, K.nx, K.ny, L.c0, L.c1, L.c2, cb, cj);
                cell_scales(L.c0, L.c1, L.c2);
                unsigned acc = 0;
                int cap_axis = -1, cap_clamp = 0;
                double cap_H = 0.0;
                const Capture capture{&cap_axis, &cap_H, &cap_clamp};
                for (;;) {
                    if (nrec == target && !last) break;
                    StepRec pre;
                    pre.p0 = L.p0, pre.p1 = L.p1, pre.p2 = L.p2;
                    pre.c0 = L.c0, pre.c1 = L.c1, pre.c2 = L.c2;
                    int fin_st = -1, fin_face = -1;
                    bool need_load = false;
                    const unsigned before = acc;
                    lane_iterate<T, TW, Capture, SCH>(L, cb, cj, K, fin_st, fin_face, need_load, acc,
                                                       capture);
                    if (acc != before) {
                        if (nrec >= target) {
                            bad = true;
                            break;
                        }
                        pre.H = cap_H;
                        pre.axis = cap_axis;
                        pre.clamp = cap_clamp;
                        buf[nrec++] = pre;
                    }
                    if (fin_st >= 0) {
                        if (fin_st != 0 || nrec != target || !last) bad = true;
                        break;
                    }
                    if (need_load) {
                        load_cell<T, S, TW>(J.nodes, K.nx, K.ny, L.c0, L.c1, L.c2, cb, cj);
                        cell_scales(L.c0, L.c1, L.c2);
                    }
                }
                if (!bad && last) {
                    // the end's adjoint into the local units of the cell it ends in
                    for (int a = 0; a < 3; a++)
                        lam[a] *= (T)(str ? 1.0 / J.iw[a][a == 0 ? L.c0 : (a == 1 ? L.c1 : L.c2)]
                                          : J.spacing[a]);
                }
                if (!bad && !last) {
                    const Ckpt nx = bp.tape[next];
                    if (nx.c0 != L.c0 || nx.c1 != L.c1 || nx.c2 != L.c2 || nx.p0 != (double)L.p0 ||
                        nx.p1 != (double)L.p1 || nx.p2 != (double)L.p2 || nx.h != (double)L.h)
                        bad = true;
                }
            }
            if (!bad) {
                // reverse sweep over the segment
                int cc0 = -1, cc1 = -1, cc2 = -1;
                for (int r = nrec - 1; r >= 0; r--) {
                    const StepRec sr = buf[r];
                    if (sr.c0 != cc0 || sr.c1 != cc1 || sr.c2 != cc2) {
                        if (cc0 >= 0) flush_cell<T, TW>(bp.gnode, nn, K.nx, K.ny, cc0, cc1, cc2, gB, gJ);
                        cc0 = sr.c0, cc1 = sr.c1, cc2 = sr.c2;
                        load_cell<T, S, TW>(J.nodes, K.nx, K.ny, cc0, cc1, cc2, cb, cj);
                        cell_scales(cc0, cc1, cc2);
                    }
                    const int endb = (last && r == nrec - 1) ? endax : -1;
                    step_adjoint<T, TW, SCH>(cb, cj, sr, K, sgn, endb, lam, ltw, gB, gJ);
                    n_steps++;
                }
                if (cc0 >= 0) flush_cell<T, TW>(bp.gnode, nn, K.nx, K.ny, cc0, cc1, cc2, gB, gJ);
                if (ck == 0 && rj == 1 && bp.lam_seed) {
                    // a rotated-S0 line's adjoint at its seed, which depends on B0 (its
                    // offset along U or V): local units -> physical
                    const int64_t lh = h - bp.nhalf0;
                    const int cs[3] = {cp.c0, cp.c1, cp.c2};
                    for (int a = 0; a < 3; a++)
                        bp.lam_seed[3 * lh + a] = (double)lam[a] * (str ? J.iw[a][cs[a]] : 1.0 / J.spacing[a]);
                }
                next = ckslot;
                ckslot = cp.prev;
                ck--;
            }
        }
        if (bad || ckslot < 0 || ck < 0) {
            if (!bad && (ck != -1 || ckslot != -1)) bad = true;  // the chain and the count disagree
            if (bad) n_bad++;
            h = -1;
        }
    }
    if (bp.stats) {
        if (n_half) atomicAdd(bp.stats + 0, n_half);
        if (n_steps) atomicAdd(bp.stats + 1, n_steps);
        if (n_bad) atomicAdd(bp.stats + 2, n_bad);
        if (n_drop) atomicAdd(bp.stats + 3, n_drop);
    }
}

// ----------------------------------------------------------------------------------
// Weight of the value at index n in the derivative at index m along one axis of N
// nodes: the second-order differences of the prep pass (central inside, one-sided
// on the boundary nodes, a plain difference when N < 3).
__device__ __forceinline__ double dcoef(int m, int n, int N, double ih)
{
    if (N < 3) return n == 1 ? ih : (n == 0 ? -ih : 0.0);
    if (m == 0) return n == 0 ? -1.5 * ih : (n == 1 ? 2.0 * ih : (n == 2 ? -0.5 * ih : 0.0));
    if (m == N - 1)
        return n == N - 1 ? 1.5 * ih : (n == N - 2 ? -2.0 * ih : (n == N - 3 ? 0.5 * ih : 0.0));
    return n == m + 1 ? 0.5 * ih : (n == m - 1 ? -0.5 * ih : 0.0);
}

// The same weight on a stretched axis with node coordinates x: the derivative of the
// quadratic through node m and its two neighbours (the two inward ones on a boundary
// node), as the prep pass takes it; a plain difference when N < 3.
__device__ __forceinline__ double dcoef_s(int m, int n, int N, const double *x)
{
    if (N < 3) {
        const double ih = 1.0 / (x[1] - x[0]);
        return n == 1 ? ih : (n == 0 ? -ih : 0.0);
    }
    const int m1 = m == 0 ? 1 : (m == N - 1 ? N - 2 : m - 1);
    const int m2 = m == 0 ? 2 : (m == N - 1 ? N - 3 : m + 1);
    const double h1 = x[m1] - x[m], h2 = x[m2] - x[m];
    const double D = h1 * h2 * (h2 - h1);
    if (n == m1) return h2 * h2 / D;
    if (n == m2) return -h1 * h1 / D;
    if (n == m) return (h1 * h1 - h2 * h2) / D;
    return 0.0;
}

// (D_axis)^T g at node (i, j, k): sum over the nodes m whose difference uses it
// (x: the axis's node coordinates on a stretched axis, else NULL)
__device__ double dT(const double *g, int axis, int i, int j, int k, int nx, int ny, int nz,
                     double ih, const double *x)
{
    const int N = axis == 0 ? nx : (axis == 1 ? ny : nz);
    const int n = axis == 0 ? i : (axis == 1 ? j : k);
    const int64_t stride = axis == 0 ? 1 : (axis == 1 ? (int64_t)nx : (int64_t)nx * ny);
    const int64_t q = ((int64_t)k * ny + j) * nx + i;
    double acc = 0.0;
    const int lo = N < 3 ? 0 : n - 2, hi = N < 3 ? N - 1 : n + 2;
    for (int m = lo; m <= hi; m++) {
        if (m < 0 || m >= N) continue;
        const double c = x ? dcoef_s(m, n, N, x) : dcoef(m, n, N, ih);
        if (c != 0.0) acc += c * g[q + (int64_t)(m - n) * stride];
    }
    return acc;
}

__global__ void grad_planes_kernel(int nx, int ny, int nz, double ihx, double ihy, double ihz,
                                   const double *cx, const double *cy, const double *cz,
                                   const double *__restrict__ gnode, int want_tw, double *gx,
                                   double *gy, double *gz)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y, k = blockIdx.z;
    if (i >= nx) return;
    const int64_t nn = (int64_t)nx * ny * nz;
    const int64_t q = ((int64_t)k * ny + j) * nx + i;
    double bx = gnode[q], by = gnode[nn + q], bz = gnode[2 * nn + q];
    if (want_tw) {
        // J = (dBz/dy - dBy/dz, dBx/dz - dBz/dx, dBy/dx - dBx/dy)
        const double *gjx = gnode + 3 * nn, *gjy = gnode + 4 * nn, *gjz = gnode + 5 * nn;
        bx += dT(gjy, 2, i, j, k, nx, ny, nz, ihz, cz) - dT(gjz, 1, i, j, k, nx, ny, nz, ihy, cy);
        by += dT(gjz, 0, i, j, k, nx, ny, nz, ihx, cx) - dT(gjx, 2, i, j, k, nx, ny, nz, ihz, cz);
        bz += dT(gjx, 1, i, j, k, nx, ny, nz, ihy, cy) - dT(gjy, 0, i, j, k, nx, ny, nz, ihx, cx);
    }
    gx[q] += bx;
    gy[q] += by;
    gz[q] += bz;
}

}  // namespace

hipError_t launch_map_backward(const MapJob &m, const double *dq, const double *dtw,
                               const double *dend_b, const double *dend_f, double *lam_end,
                               double *lam_tw, double *gnode, int64_t nhalf0, hipStream_t s)
{
    const int64_t np = m.nu * m.nv * m.nlayers;
    int64_t b = (np + 255) / 256;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    hipLaunchKernelGGL(map_backward_kernel, dim3((unsigned)b), dim3(256), 0, s, m, dq, dtw, dend_b,
                       dend_f, lam_end, lam_tw, gnode, nhalf0);
    return hipGetLastError();
}

namespace {
// A rotated S0's four lines start at r0 -+ delta U and r0 -+ delta V, with U the
// normalised e_a x b (e_a the axis least aligned with b = B0/|B0|, held fixed) and
// V = b x U: their seed adjoints (both halves of each line) give dL/dU and dL/dV,
// taken back through V = b x U, U = w/|w|, w = e_a x b and b = B0/|B0| to dL/dB0,
// which goes to the nodes by the FP64 trilinear weights at r0.
__global__ void rot_seed_kernel(MapJob m, const RotEntry *__restrict__ rot,
                                const uint32_t *__restrict__ rot_count, int64_t cap,
                                const double *__restrict__ lam_seed, double *gnode)
{
    const int64_t nn = (int64_t)m.n[0] * m.n[1] * m.n[2];
    int64_t cnt = (int64_t)*rot_count;
    if (cnt > cap) cnt = cap;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cnt;
         e += (int64_t)gridDim.x * blockDim.x) {
        const RotEntry E = rot[e];
        double lk[4][3];
        for (int k = 0; k < 4; k++) {
            const int64_t line = 4 * e + k;
            for (int a = 0; a < 3; a++)
                lk[k][a] = lam_seed[3 * line + a] + lam_seed[3 * (m.rot_nlines + line) + a];
        }
        double gU[3], gV[3];
        for (int a = 0; a < 3; a++) {
            gU[a] = m.rot_delta * (lk[1][a] - lk[0][a]);
            gV[a] = m.rot_delta * (lk[3][a] - lk[2][a]);
        }
        if (gU[0] == 0.0 && gU[1] == 0.0 && gU[2] == 0.0 && gV[0] == 0.0 && gV[1] == 0.0 && gV[2] == 0.0)
            continue;
        double B[3];
        field64(m, E.r0, B);
        const double bm = sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
        const double b[3] = {B[0] / bm, B[1] / bm, B[2] / bm};
        int ax = 0;
        if (fabs(b[1]) < fabs(b[ax])) ax = 1;
        if (fabs(b[2]) < fabs(b[ax])) ax = 2;
        const double *U = E.U;
        // V = b x U: dL/db += U x gV, dL/dU += gV x b
        double gb[3] = {U[1] * gV[2] - U[2] * gV[1], U[2] * gV[0] - U[0] * gV[2], U[0] * gV[1] - U[1] * gV[0]};
        const double gu[3] = {gU[0] + gV[1] * b[2] - gV[2] * b[1], gU[1] + gV[2] * b[0] - gV[0] * b[2],
                              gU[2] + gV[0] * b[1] - gV[1] * b[0]};
        // U = w / |w|, w = e_ax x b
        double w[3] = {0.0, 0.0, 0.0};
        if (ax == 0) w[1] = -b[2], w[2] = b[1];
        else if (ax == 1) w[0] = b[2], w[2] = -b[0];
        else w[0] = -b[1], w[1] = b[0];
        const double wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        const double uu = U[0] * gu[0] + U[1] * gu[1] + U[2] * gu[2];
        double gw[3];
        for (int a = 0; a < 3; a++) gw[a] = (gu[a] - U[a] * uu) / wn;
        // w = e_ax x b: dL/db += gw x e_ax
        if (ax == 0) gb[1] += gw[2], gb[2] -= gw[1];
        else if (ax == 1) gb[0] -= gw[2], gb[2] += gw[0];
        else gb[0] += gw[1], gb[1] -= gw[0];
        // b = B0 / |B0|
        const double bb = b[0] * gb[0] + b[1] * gb[1] + b[2] * gb[2];
        Tri t;
        tri_of(m, E.r0, t);
        for (int c = 0; c < 3; c++) {
            const double gB = (gb[c] - b[c] * bb) / bm;
            if (gB == 0.0) continue;
            for (int q = 0; q < 8; q++) atomicAdd(gnode + c * nn + t.node[q], gB * t.w[q]);
        }
    }
}
}  // namespace

hipError_t launch_rot_seed(const MapJob &m, const RotEntry *rot, const uint32_t *rot_count,
                           int64_t cap, const double *lam_seed, double *gnode, hipStream_t s)
{
    int64_t b = (cap + 255) / 256;
    if (b < 1) b = 1;
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(rot_seed_kernel, dim3((unsigned)b), dim3(256), 0, s, m, rot, rot_count, cap,
                       lam_seed, gnode);
    return hipGetLastError();
}

namespace {

__global__ void bwd_key_kernel(const int32_t *__restrict__ tape_acc, int64_t n,
                               int32_t *__restrict__ key)
{
    for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < n;
         h += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = tape_acc[h];
        key[h] = a <= 0 ? 0 : (a >= 1020 ? 255 : a >> 2);
    }
}

}  // namespace

hipError_t launch_bwd_order(const int32_t *tape_acc, int64_t nhalves, int32_t *key,
                            uint32_t *counts, int32_t *order, hipStream_t s)
{
    int64_t b = (nhalves + 255) / 256;
    if (b < 1) b = 1;
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(bwd_key_kernel, dim3((unsigned)b), dim3(256), 0, s, tape_acc, nhalves, key);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_bucket_order(nhalves, key, counts, order, s);
}

namespace {
// FP64 records: the all-FP64 form; FP32 records: the F32X form, whose forward pass and
// so its replay and reverse sweep are FP32
template <int SCH>
void launch_bwd_s(int store, int want_tw, const TraceJob *job_dev, const BwdParams &bp, hipStream_t s)
{
    const dim3 grid((unsigned)((bp.nslots + 63) / 64)), blk(64);
    if (store == FQ_DT_F64) {
        if (want_tw) hipLaunchKernelGGL((trace_backward_kernel<double, double, true, SCH>), grid, blk, 0, s, job_dev, bp);
        else hipLaunchKernelGGL((trace_backward_kernel<double, double, false, SCH>), grid, blk, 0, s, job_dev, bp);
    } else {
        if (want_tw) hipLaunchKernelGGL((trace_backward_kernel<float, float, true, SCH>), grid, blk, 0, s, job_dev, bp);
        else hipLaunchKernelGGL((trace_backward_kernel<float, float, false, SCH>), grid, blk, 0, s, job_dev, bp);
    }
}
}  // namespace

hipError_t launch_trace_backward(int store, int want_tw, const TraceJob *job_dev,
                                 const BwdParams &bp, hipStream_t s)
{
    if (bp.scheme == SCH_RKF45) launch_bwd_s<SCH_RKF45>(store, want_tw, job_dev, bp, s);
    else if (bp.scheme == SCH_RK4) launch_bwd_s<SCH_RK4>(store, want_tw, job_dev, bp, s);
    else if (bp.scheme == SCH_RK4_38) launch_bwd_s<SCH_RK4_38>(store, want_tw, job_dev, bp, s);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_grad_planes(const fq_field &f, const double *gnode, int want_tw,
                              double *const gb[3], hipStream_t s)
{
    const unsigned bxs = (unsigned)((f.n[0] + 255) / 256);
    hipLaunchKernelGGL(grad_planes_kernel, dim3(bxs, (unsigned)f.n[1], (unsigned)f.n[2]), dim3(256),
                       0, s, (int)f.n[0], (int)f.n[1], (int)f.n[2], 1.0 / f.spacing[0],
                       1.0 / f.spacing[1], 1.0 / f.spacing[2], f.coord[0], f.coord[1], f.coord[2],
                       gnode, want_tw, gb[0], gb[1], gb[2]);
    return hipGetLastError();
}

}  // namespace fq
