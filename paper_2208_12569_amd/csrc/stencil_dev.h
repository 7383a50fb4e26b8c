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
        P.coord[a] = m.coord[a];
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

// (selects between fixed elements: an index computed at run time would put the
// caller's arrays in scratch memory)
__device__ __forceinline__ void inface(int face, const double e[3], double uv[2])
{
    const int a = face >> 1;
    uv[0] = a == 0 ? e[1] : e[0];
    uv[1] = a == 2 ? e[1] : e[2];
}

// component a (0, 1, 2) of v, by selects
__device__ __forceinline__ double comp3(const double v[3], int a)
{
    return a == 0 ? v[0] : (a == 1 ? v[1] : v[2]);
}

__device__ __forceinline__ bool edge_end(const MapJob &m, int face, const double e[3])
{
    if (face < 0) return false;
    const int a = face >> 1;
    for (int b = 0; b < 3; b++) {
        if (b == a) continue;
        const double lo = axis_lo(m, b), hi = axis_hi(m, b);
        if (e[b] - lo < m.edge_eps || hi - e[b] < m.edge_eps) return true;
    }
    return false;
}

// A neighbour line as the stencil needs it: the in-face coordinates of its S1 and S2
// ends, their faces, its status, which half is S1 and whether an end lies near a box
// edge. Kept small so that a point and its four neighbours stay in registers.
struct Nb {
    double u1[2], u2[2];
    int f1, f2;
    uint16_t st;
    bool swapped, edge;
};

__device__ __forceinline__ Nb read_nb(const MapJob &m, const HalfRecs &R, int64_t nlines, int64_t l)
{
    Line L;
    read_line(R, nlines, l, L);
    Nb n;
    inface(L.f1, L.e1, n.u1);
    inface(L.f2, L.e2, n.u2);
    n.f1 = L.f1;
    n.f2 = L.f2;
    n.st = L.st;
    n.swapped = L.swapped;
    n.edge = edge_end(m, L.f1, L.e1) || edge_end(m, L.f2, L.e2);
    return n;
}

// Which difference an S0 axis takes: central where both neighbours end on the
// centre line's faces at both ends, else one-sided with the neighbour that does.
enum AxisRule { RULE_NONE = 0, RULE_CENTRAL, RULE_PLUS, RULE_MINUS };

__device__ __forceinline__ bool usable(const Line &c, const Nb &o, bool present)
{
    return present && !(o.st & kFatal) && o.f1 == c.f1 && o.f2 == c.f2;
}

// mn / pn: the neighbours on the minus / plus side, hm / hp: whether they exist
__device__ __forceinline__ int axis_rule(const Line &c, const Nb &mn, bool hm, const Nb &pn, bool hp)
{
    const bool um = usable(c, mn, hm), up = usable(c, pn, hp);
    if (um && up) return RULE_CENTRAL;
    if (up) return RULE_PLUS;
    if (um) return RULE_MINUS;
    return RULE_NONE;
}

// derivatives of (u1, v1) and (u2, v2) along one S0 axis by the given rule (not
// RULE_NONE); c1, c2: the centre line's in-face coordinates
__device__ __forceinline__ void axis_diff(int rule, const double c1[2], const double c2[2],
                                          const Nb &mn, const Nb &pn, double d, double d1[2],
                                          double d2[2], uint16_t &st)
{
    if (rule == RULE_CENTRAL) {
        const double s = 0.5 / d;
        for (int q = 0; q < 2; q++) {
            d1[q] = (pn.u1[q] - mn.u1[q]) * s;
            d2[q] = (pn.u2[q] - mn.u2[q]) * s;
        }
        return;
    }
    const bool up = rule == RULE_PLUS;
    const double s = 1.0 / d;
    for (int q = 0; q < 2; q++) {
        d1[q] = up ? (pn.u1[q] - c1[q]) * s : (c1[q] - mn.u1[q]) * s;
        d2[q] = up ? (pn.u2[q] - c2[q]) * s : (c2[q] - mn.u2[q]) * s;
    }
    st |= FQ_ST_ONESIDED;
}

__device__ __forceinline__ void point_pos(const MapJob &m, int64_t i, int64_t j, int64_t k, double r[3])
{
    for (int a = 0; a < 3; a++)
        r[a] = m.p_origin[a] + (double)i * m.p_a[a] + (double)j * m.p_b[a] + (double)k * m.p_c[a];
}

}  // namespace sten
}  // namespace fq
