// Map-assembly helpers shared by the Q stencil and its adjoint: half-line records
// read back as lines with ends ordered S1, S2, in-face coordinates, and the
// stencil rule.
#pragma once

#include <math.h>

#include "fq_internal.h"

namespace fq {
namespace sten {

constexpr uint16_t kFatal = FQ_ST_OUTSIDE | FQ_ST_NULLB | FQ_ST_MAXSTEPS | FQ_ST_NONFINITE;

__device__ __forceinline__ void field64(const MapJob &m, const double r[3], double B[3])
{
    Planes64 P;
    for (int a = 0; a < 3; a++) {
        P.b[a] = m.b[a];
        P.n[a] = m.n[a];
        P.origin[a] = m.origin[a];
        P.spacing[a] = m.spacing[a];
    }
    P.dtype = m.dtype;
    interp64(P, r, B);
}

// One line read back from the half records, with its ends ordered as S1, S2.
struct Line {
    double e1[3], e2[3];
    int f1, f2;
    uint16_t st;
    double tw, len;
    bool swapped;  // S1 is the forward end
};

__device__ __forceinline__ void read_line(const HalfRecs &R, int64_t nlines, int64_t l, Line &L)
{
    const int64_t hb = l, hf = nlines + l;
    const double lb = R.len[hb], lf = R.len[hf];
    L.st = R.st[hb] | R.st[hf];
    L.tw = R.tw[hb] + R.tw[hf];
    L.len = lb + lf;
    L.swapped = (lf == 0.0 && lb != 0.0);
    const int64_t s1 = L.swapped ? hf : hb, s2 = L.swapped ? hb : hf;
    for (int a = 0; a < 3; a++) {
        L.e1[a] = R.end[3 * s1 + a];
        L.e2[a] = R.end[3 * s2 + a];
    }
    L.f1 = R.face[s1];
    L.f2 = R.face[s2];
}

__device__ __forceinline__ void inface(int face, const double e[3], double uv[2])
{
    const int a = face >> 1;
    uv[0] = e[a == 0 ? 1 : 0];
    uv[1] = e[a == 2 ? 1 : 2];
}

__device__ __forceinline__ bool edge_end(const MapJob &m, int face, const double e[3])
{
    if (face < 0) return false;
    const int a = face >> 1;
    for (int b = 0; b < 3; b++) {
        if (b == a) continue;
        const double lo = m.origin[b], hi = m.origin[b] + (m.n[b] - 1) * m.spacing[b];
        if (e[b] - lo < m.edge_eps || hi - e[b] < m.edge_eps) return true;
    }
    return false;
}

__device__ __forceinline__ bool usable(const Line &c, const Line &o)
{
    return !(o.st & kFatal) && o.f1 == c.f1 && o.f2 == c.f2;
}

// Which difference an S0 axis takes: central where both neighbours end on the
// centre line's faces at both ends, else one-sided with the neighbour that does.
enum AxisRule { RULE_NONE = 0, RULE_CENTRAL, RULE_PLUS, RULE_MINUS };

__device__ __forceinline__ int axis_rule(const Line &c, const Line *m, const Line *p)
{
    const bool um = m && usable(c, *m), up = p && usable(c, *p);
    if (um && up) return RULE_CENTRAL;
    if (up) return RULE_PLUS;
    if (um) return RULE_MINUS;
    return RULE_NONE;
}

// derivatives of (u1, v1) and (u2, v2) along one S0 axis; false if no neighbour fits
__device__ __forceinline__ bool axis_diff(const Line &c, const Line *m, const Line *p, double d, double d1[2],
                          double d2[2], uint16_t &st)
{
    const int rule = axis_rule(c, m, p);
    if (rule == RULE_NONE) return false;
    double c1[2], c2[2], a1[2], a2[2], b1[2], b2[2];
    inface(c.f1, c.e1, c1);
    inface(c.f2, c.e2, c2);
    if (rule != RULE_PLUS) {
        inface(m->f1, m->e1, a1);
        inface(m->f2, m->e2, a2);
    }
    if (rule != RULE_MINUS) {
        inface(p->f1, p->e1, b1);
        inface(p->f2, p->e2, b2);
    }
    if (rule == RULE_CENTRAL) {
        const double s = 0.5 / d;
        for (int q = 0; q < 2; q++) {
            d1[q] = (b1[q] - a1[q]) * s;
            d2[q] = (b2[q] - a2[q]) * s;
        }
        return true;
    }
    const bool up = rule == RULE_PLUS;
    const double s = 1.0 / d;
    for (int q = 0; q < 2; q++) {
        d1[q] = up ? (b1[q] - c1[q]) * s : (c1[q] - a1[q]) * s;
        d2[q] = up ? (b2[q] - c2[q]) * s : (c2[q] - a2[q]) * s;
    }
    st |= FQ_ST_ONESIDED;
    return true;
}

__device__ __forceinline__ void point_pos(const MapJob &m, int64_t i, int64_t j, int64_t k, double r[3])
{
    for (int a = 0; a < 3; a++)
        r[a] = m.p_origin[a] + (double)i * m.p_a[a] + (double)j * m.p_b[a] + (double)k * m.p_c[a];
}

}  // namespace sten
}  // namespace fq
