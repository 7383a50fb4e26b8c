// Per-lane stepping logic of the field-line tracer (host + device).
//
// One call of lane_iterate() makes one trial step of one half line inside its
// current grid cell; the caller owns the cell coefficients and refetches them when
// the call reports a cell change. The same function runs in the tracer kernel and
// in the adjoint's replays of recorded segments (which capture the accepted steps
// through the event sink).
//
// Method: RKF45 (Fehlberg's 4(5) pair, fifth-order solution kept; Section 2.3) on
// dr/ds = B/|B| (Section 2.1, Eq. rb) with the Eq. tw integrand (Section 1) and the
// length as extra components. B and curl B come from the cell's trilinear
// interpolant (Section 2.2, Eq. interp) in monomial form. Position = cell index +
// local coordinates in [0,1]. A step whose straight-line guess reaches a face is
// taken with that face's normal coordinate as the independent variable, so it ends
// exactly on the face.
#pragma once

#include <float.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace fq {

template <typename T> struct Num;
template <> struct Num<float> {
    static __host__ __device__ __forceinline__ float fma_(float a, float b, float c)
    {
        return __builtin_fmaf(a, b, c);
    }
    static __host__ __device__ __forceinline__ float rsq(float x)
    {
#if defined(__HIP_DEVICE_COMPILE__)
        return __builtin_amdgcn_rsqf(x);
#else
        return 1.0f / sqrtf(x);
#endif
    }
    static __host__ __device__ __forceinline__ float rcp(float x)
    {
#if defined(__HIP_DEVICE_COMPILE__)
        return __builtin_amdgcn_rcpf(x);
#else
        return 1.0f / x;
#endif
    }
    static constexpr float ov = 1e-5f;        // overshoot of a step past a face that is kept
    // Method II: the gradient of the trilinear B/B jumps across a cell face, so an
    // overshoot d kept there moves U and V by d times that jump (first order, where
    // positions err by d^2): about two ulp of a local coordinate
    static constexpr float ov_tan = 1.2e-7f;
    static constexpr float tau = 1e-4f;       // |direction component| below this is tangent
    static constexpr float null_rel = 1e-30f; // |B|^2 below null_rel * max|B|^2 is a null
    static constexpr float gmin = 1e-4f;      // smallest usable d(coordinate)/ds on a landing
    static constexpr float hmin = 1e-6f;      // smallest plain step (reference lengths)
};
template <> struct Num<double> {
    static __host__ __device__ __forceinline__ double fma_(double a, double b, double c)
    {
        return __builtin_fma(a, b, c);
    }
    // 1/sqrt(x) and 1/x: the hardware estimates (relative error about 5e-8) refined
    // by one Newton-Raphson iteration each (to about 5e-15 relative, measured on
    // gfx950) instead of the IEEE division and square root sequences. Arguments are
    // positive normal |B|^2 values and direction components bounded away from zero
    // by the callers.
    static __host__ __device__ __forceinline__ double rsq(double x)
    {
#if defined(__HIP_DEVICE_COMPILE__)
        const double y = __builtin_amdgcn_rsq(x);
        return y * __builtin_fma(-0.5 * x * y, y, 1.5);
#else
        return 1.0 / sqrt(x);
#endif
    }
    static __host__ __device__ __forceinline__ double rcp(double x)
    {
#if defined(__HIP_DEVICE_COMPILE__)
        const double y = __builtin_amdgcn_rcp(x);
        return __builtin_fma(y, __builtin_fma(-x, y, 1.0), y);
#else
        return 1.0 / x;
#endif
    }
    static constexpr double ov = 1e-9;
    static constexpr double ov_tan = 1e-9;
    static constexpr double tau = 1e-9;
    static constexpr double null_rel = 1e-60;
    static constexpr double gmin = 1e-9;
    static constexpr double hmin = 1e-12;
};

// x^(1/10) for the step controller, which works on squared errors (accuracy of a
// few ulp is plenty: it only scales the next trial step)
__host__ __device__ __forceinline__ float pow01(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_exp2f(0.1f * __builtin_amdgcn_logf(x));
#else
    return powf(x, 0.1f);
#endif
}

template <typename T> __host__ __device__ __forceinline__ T mn(T a, T b) { return a < b ? a : b; }
template <typename T> __host__ __device__ __forceinline__ T mx(T a, T b) { return a > b ? a : b; }
template <typename T> __host__ __device__ __forceinline__ bool finite_(T x)
{
    return __builtin_isfinite(x);
}
template <typename T> __host__ __device__ __forceinline__ T sel3(int a, T x, T y, T z)
{
    return a == 0 ? x : (a == 1 ? y : z);
}

// P(u,v,w) = c0 + c1 u + c2 v + c3 w + c4 uv + c5 uw + c6 vw + c7 uvw, 7 FMAs.
template <typename T>
__host__ __device__ __forceinline__ T poly(const T c[8], T u, T v, T w)
{
    using N = Num<T>;
    T a = N::fma_(c[5], w, c[1]);
    T b = N::fma_(c[6], w, c[2]);
    T d = N::fma_(c[7], w, c[4]);
    T e = N::fma_(c[3], w, c[0]);
    b = N::fma_(u, d, b);
    e = N::fma_(u, a, e);
    return N::fma_(v, b, e);
}

// Monomial coefficients from the 8 corner values f[x + 2y + 4z].
template <typename T>
__host__ __device__ __forceinline__ void coeffs(const T f[8], T c[8])
{
    c[0] = f[0];
    c[1] = f[1] - f[0];
    c[2] = f[2] - f[0];
    c[3] = f[4] - f[0];
    c[4] = (f[3] - f[1]) - (f[2] - f[0]);
    c[5] = (f[5] - f[1]) - (f[4] - f[0]);
    c[6] = (f[6] - f[2]) - (f[4] - f[0]);
    c[7] = ((f[7] - f[6]) - (f[5] - f[4])) - ((f[3] - f[2]) - (f[1] - f[0]));
}

// Direction (local units per reference length), twist integrand per reference
// length and |B|^2 at local point (u,v,w).
template <typename T, bool TW>
__host__ __device__ __forceinline__ void rhs(const T cb[3][8], const T cj[3][8], T u, T v, T w,
                                             T sgn, T rx, T ry, T rz, T twk, T &f0, T &f1, T &f2,
                                             T &ft, T &b2)
{
    using N = Num<T>;
    const T bx = poly<T>(cb[0], u, v, w);
    const T by = poly<T>(cb[1], u, v, w);
    const T bz = poly<T>(cb[2], u, v, w);
    b2 = N::fma_(bx, bx, N::fma_(by, by, bz * bz));
    const T inv = N::rsq(b2);
    const T s = sgn * inv;
    f0 = s * bx * rx;
    f1 = s * by * ry;
    f2 = s * bz * rz;
    if (TW) {
        const T jx = poly<T>(cj[0], u, v, w);
        const T jy = poly<T>(cj[1], u, v, w);
        const T jz = poly<T>(cj[2], u, v, w);
        const T jb = N::fma_(jx, bx, N::fma_(jy, by, jz * bz));
        ft = jb * (inv * inv) * twk;
    } else {
        ft = T(0);
    }
}

// State of one half line.
template <typename T> struct Lane {
    int c0, c1, c2;  // cell
    T p0, p1, p2;    // local coordinates in [0,1]
    T h, tol, sgn;   // step (reference lengths), error bound (grid spacings), direction
    double tw, len;  // twist and length (reference lengths) so far
    int64_t trials;
    int force;       // 2*axis + (direction > 0) of a landing to try next, -1 = none
};

template <typename T> struct LaneConst {
    T rx, ry, rz;    // reference length / spacing per axis
    T twk;           // reference length / (4 pi)
    T bnull2;        // null-field threshold on |B|^2
    int nx, ny, nz;  // nodes per axis
    int64_t max_steps;
};

// Method II (Section 2.1, Eq. rb2): the two tangent vectors U, V carried along the
// line, in local grid units (component a in units of the spacing of axis a), so
// that dU/ds = J U with J the Jacobian of the local direction field
// f = sgn R B/|B| (R = diag(rx, ry, rz)) with respect to the local coordinates.
template <typename T> struct Tan {
    T u[3], v[3];
};

// d/du, d/dv, d/dw of the cell polynomial P (see poly).
template <typename T>
__host__ __device__ __forceinline__ void dpoly(const T c[8], T u, T v, T w, T &du, T &dv, T &dw)
{
    using N = Num<T>;
    du = N::fma_(v, N::fma_(c[7], w, c[4]), N::fma_(c[5], w, c[1]));
    dv = N::fma_(u, N::fma_(c[7], w, c[4]), N::fma_(c[6], w, c[2]));
    dw = N::fma_(u, N::fma_(c[7], v, c[5]), N::fma_(c[6], v, c[3]));
}

// The rates of U and V at local point (u,v,w), per reference length: J U and J V
// with J = sgn R (I - b b^T) (dB/dp) / |B| and b = B/|B| (B given, inv = 1/|B|).
// The gradient of B/B is taken analytically on the cell's interpolant.
template <typename T>
__host__ __device__ __forceinline__ void tan_rates(const T cb[3][8], T u, T v, T w, T bx, T by,
                                                   T bz, T inv, T sgn, T rx, T ry, T rz,
                                                   const T U[3], const T V[3], T kU[3], T kV[3])
{
    using N = Num<T>;
    T d[3][3];  // d[i][j] = dB_i / dp_j
#pragma unroll
    for (int i = 0; i < 3; i++) dpoly<T>(cb[i], u, v, w, d[i][0], d[i][1], d[i][2]);
    const T b0 = bx * inv, b1 = by * inv, b2 = bz * inv;
    const T s = sgn * inv;
#pragma unroll
    for (int m = 0; m < 2; m++) {
        const T *X = m ? V : U;
        T *K = m ? kV : kU;
        T g[3];
#pragma unroll
        for (int i = 0; i < 3; i++) g[i] = N::fma_(d[i][0], X[0], N::fma_(d[i][1], X[1], d[i][2] * X[2]));
        const T bg = N::fma_(b0, g[0], N::fma_(b1, g[1], b2 * g[2]));
        K[0] = s * rx * N::fma_(-b0, bg, g[0]);
        K[1] = s * ry * N::fma_(-b1, bg, g[1]);
        K[2] = s * rz * N::fma_(-b2, bg, g[2]);
    }
}

// Why a trial ended (an event sink may record it; the tracer ignores it).
enum Ev : int {
    EV_CROSS = 0,     // moved to the next cell through the face it sat on
    EV_NOLAND,        // a landing was not possible yet: plain step next
    EV_REJECT_ARC,    // plain step over the error bound
    EV_REJECT_LAND,   // landing over the error bound
    EV_ACCEPT_ARC,    // plain step accepted
    EV_CURVED_OUT,    // plain step left the cell by more than ov
    EV_LAND_OTHER,    // landing left through another face first
    EV_LAND_BREAK,    // landing parametrisation broke down
    EV_ACCEPT_LAND,   // landing accepted
    EV_COUNT
};

struct NoEvents {
    __host__ __device__ __forceinline__ void operator()(int) const {}
    // an accepted step: landing axis (-1 for a plain step), its signed length in the
    // independent variable (arc length for a plain step, the axis coordinate for a
    // landing) and the coordinates (bit q) it left past a box face and that were
    // clamped onto it
    template <typename T> __host__ __device__ __forceinline__ void accepted(int, T, int) const {}
};

// Carry a coordinate that left [0,1] by a small amount into the neighbouring cell
// (on a box face it is clamped to the face, and `bit` is set in `clamped`). Returns
// true if the cell changed.
template <typename T>
__host__ __device__ __forceinline__ bool carry(int &c, T &p, int n, int &clamped, int bit)
{
    if (p > T(1)) {
        if (c < n - 2) {
            c++;
            p -= T(1);
            return true;
        }
        p = T(1);
        clamped |= bit;
    } else if (p < T(0)) {
        if (c > 0) {
            c--;
            p += T(1);
            return true;
        }
        p = T(0);
        clamped |= bit;
    }
    return false;
}

// Did the step leave [-ov, 1+ov] along this axis and come back? The coordinate
// along the step is modelled by the quadratic through its start (slope s1 = H k1)
// and its end (displacement D); returns the face code 2*axis + (high side) of an
// interior extremum beyond the cell, or -1.
template <typename T>
__host__ __device__ __forceinline__ int excursion(int axis, T p, T s1, T D, T ov)
{
    // x(t) = p + s1 t + s2 t^2 on t in [0,1]; an interior extremum needs s1 s2 < 0 and
    // t* = -s1 / (2 s2) < 1, and lies at x* = p - s1^2 / (4 s2). Written without
    // divisions: with a = |s2| the conditions are |s1| < 2a and, for a maximum
    // (s2 < 0), s1^2 > 4a (1 + ov - p); for a minimum, s1^2 > 4a (p + ov).
    const T s2 = D - s1;
    if (!(s1 * s2 < T(0))) return -1;
    const T a = fabs(s2);
    if (!(fabs(s1) < T(2) * a)) return -1;
    const T s1s = s1 * s1, a4 = T(4) * a;
    if (s2 < T(0)) return s1s > a4 * (T(1) + ov - p) ? 2 * axis + 1 : -1;
    return s1s > a4 * (p + ov) ? 2 * axis : -1;
}

// Face code of a box face that a step ended past (coordinate n of cell c on an axis
// of `nodes` nodes, face codes lo and lo + 1) while the line crosses it: its
// direction component heads out through the face more steeply than gmin at the
// start of the step (d0) or at its end (d1); -1 if none. Only a line tangent to
// the face at both ends keeps the overshoot allowance: a line that turns over
// within the step and leaves at a small angle alpha would otherwise be clamped
// onto the face up to ov / alpha away from its crossing (near a polarity
// inversion line on a box face, alpha is the seed's distance from that line).
template <typename T>
__host__ __device__ __forceinline__ int box_past(T n, int c, int nodes, T d0, T d1, int lo)
{
    if (c == 0 && n < T(0) && (d0 < -Num<T>::gmin || d1 < -Num<T>::gmin)) return lo;
    if (c == nodes - 2 && n > T(1) && (d0 > Num<T>::gmin || d1 > Num<T>::gmin)) return lo + 1;
    return -1;
}

// One trial step. On return: fin_st >= 0 if the half line ended (status bits,
// fin_face = exit face or -1), need_load if the cell changed. n_acc counts
// accepted steps.
// Integration schemes (Section 2.3). RKF45 is adaptive; the two RK4 rules take a
// fixed step (L.tol holds it; the error bound is not used), cut short only by cell
// faces like every step here.
enum Scheme : int { SCH_RKF45 = 0, SCH_RK4 = 1, SCH_RK4_38 = 2 };

// M2: carry Method II's tangent vectors tn along (RKF45 only).
template <typename T, bool TW, typename EvSink = NoEvents, int SCH = SCH_RKF45, bool M2 = false>
__host__ __device__ __forceinline__ void lane_iterate(Lane<T> &L, const T cb[3][8],
                                                      const T cj[3][8], const LaneConst<T> &K,
                                                      int &fin_st, int &fin_face, bool &need_load,
                                                      unsigned &n_acc, EvSink ev = EvSink(),
                                                      Tan<T> *tn = nullptr)
{
    static_assert(!M2 || SCH == 0, "Method II is traced with RKF45");
    constexpr bool FIXED = SCH != SCH_RKF45;
    constexpr int NS = FIXED ? 4 : 6;  // stages
    using N = Num<T>;
    constexpr int kNull = 2, kMaxSteps = 4, kNonFinite = 8;  // FQ_ST_* bits
    if (++L.trials > K.max_steps) {
        fin_st = kMaxSteps;
        return;
    }
    T f0, f1, f2, ft, b2;
    rhs<T, TW>(cb, cj, L.p0, L.p1, L.p2, L.sgn, K.rx, K.ry, K.rz, K.twk, f0, f1, f2, ft, b2);
    if (!finite_(b2)) {
        fin_st = kNonFinite;
        return;
    }
    if (b2 <= K.bnull2) {
        fin_st = kNull;
        return;
    }
    // A point on a face of its cell, moving out through it, changes cell first (on a
    // box face the line ends). Between two cells a direction within tau of the
    // face plane counts as tangent: the two cells' polynomials agree on the face only
    // to rounding, so the sign of a tiny normal component may differ between them.
    // On a box face the sign alone decides, as for the exact line.
    const T tau = N::tau;
    const T th0 = L.c0 == K.nx - 2 ? T(0) : tau, tl0 = L.c0 == 0 ? T(0) : tau;
    const T th1 = L.c1 == K.ny - 2 ? T(0) : tau, tl1 = L.c1 == 0 ? T(0) : tau;
    const T th2 = L.c2 == K.nz - 2 ? T(0) : tau, tl2 = L.c2 == 0 ? T(0) : tau;
    int xa = -1, xd = 0;
    if (L.p0 == T(1) && f0 > th0) xa = 0, xd = 1;
    else if (L.p0 == T(0) && f0 < -tl0) xa = 0, xd = -1;
    else if (L.p1 == T(1) && f1 > th1) xa = 1, xd = 1;
    else if (L.p1 == T(0) && f1 < -tl1) xa = 1, xd = -1;
    else if (L.p2 == T(1) && f2 > th2) xa = 2, xd = 1;
    else if (L.p2 == T(0) && f2 < -tl2) xa = 2, xd = -1;
    if (xa >= 0) ev(EV_CROSS);
    if (xa < 0) {
        // straight-line distance to the faces ahead
        T t_exit = T(FLT_MAX);
        int a_star = -1;
        if (fabs(f0) > tau) {
            const T t = (f0 > 0 ? (T(1) - L.p0) : -L.p0) * N::rcp(f0);
            if (t < t_exit) t_exit = t, a_star = 0;
        }
        if (fabs(f1) > tau) {
            const T t = (f1 > 0 ? (T(1) - L.p1) : -L.p1) * N::rcp(f1);
            if (t < t_exit) t_exit = t, a_star = 1;
        }
        if (fabs(f2) > tau) {
            const T t = (f2 > 0 ? (T(1) - L.p2) : -L.p2) * N::rcp(f2);
            if (t < t_exit) t_exit = t, a_star = 2;
        }
        int axis = L.h >= t_exit ? a_star : -1;
        int want = 0;
        if (L.force >= 0) {
            axis = L.force >> 1;
            want = (L.force & 1) ? 1 : -1;
        }
        L.force = -1;
        T H = L.h, g0 = T(1);
        if (axis >= 0) {
            const T pa = sel3(axis, L.p0, L.p1, L.p2);
            g0 = sel3(axis, f0, f1, f2);
            H = (g0 > 0) ? (T(1) - pa) : -pa;
            const bool wrong_way = want != 0 && (g0 > 0 ? 1 : -1) != want;
            if (wrong_way || !(fabs(g0) > N::gmin) || H == T(0)) {
                // not heading to that face yet: approach it with a plain step
                L.h = mx(T(0.5) * mn(L.h, t_exit), N::hmin);
                ev(EV_NOLAND);
                return;
            }
        }
        const T hs = H >= 0 ? T(1) : T(-1);
        const T ig0 = N::rcp(g0);

        // Fehlberg 4(5), or classic / 3/8-rule RK4 (Kutta). Stage positions need only
        // the position parts of earlier stages; the twist and length parts go straight
        // into the weighted sums of the solution.
        constexpr T A10 = T(1.0 / 4.0);
        constexpr T A20 = T(3.0 / 32.0), A21 = T(9.0 / 32.0);
        constexpr T A30 = T(1932.0 / 2197.0), A31 = T(-7200.0 / 2197.0), A32 = T(7296.0 / 2197.0);
        constexpr T A40 = T(439.0 / 216.0), A41 = T(-8.0), A42 = T(3680.0 / 513.0),
                    A43 = T(-845.0 / 4104.0);
        constexpr T A50 = T(-8.0 / 27.0), A51 = T(2.0), A52 = T(-3544.0 / 2565.0),
                    A53 = T(1859.0 / 4104.0), A54 = T(-11.0 / 40.0);
        constexpr T B0 = T(16.0 / 135.0), B2 = T(6656.0 / 12825.0), B3 = T(28561.0 / 56430.0),
                    B4 = T(-9.0 / 50.0), B5 = T(2.0 / 55.0);
        constexpr T E0 = T(1.0 / 360.0), E2 = T(-128.0 / 4275.0), E3 = T(-2197.0 / 75240.0),
                    E4 = T(1.0 / 50.0), E5 = T(2.0 / 55.0);
        // classic RK4: c = (0, 1/2, 1/2, 1), b = (1, 2, 2, 1) / 6;
        // 3/8 rule: c = (0, 1/3, 2/3, 1), a = (1/3; -1/3, 1; 1, -1, 1), b = (1, 3, 3, 1) / 8
        constexpr T W0 = SCH == SCH_RK4 ? T(1.0 / 6.0) : SCH == SCH_RK4_38 ? T(1.0 / 8.0) : B0;
        T k[6][3];
        k[0][0] = f0 * ig0;
        k[0][1] = f1 * ig0;
        k[0][2] = f2 * ig0;
        T ku[M2 ? 6 : 1][3], kv[M2 ? 6 : 1][3];
        if constexpr (M2) {
            // the rates at the start need B there; one more evaluation of it
            const T bx = poly<T>(cb[0], L.p0, L.p1, L.p2), by = poly<T>(cb[1], L.p0, L.p1, L.p2),
                    bz = poly<T>(cb[2], L.p0, L.p1, L.p2);
            tan_rates<T>(cb, L.p0, L.p1, L.p2, bx, by, bz, N::rsq(b2), L.sgn, K.rx, K.ry, K.rz,
                         tn->u, tn->v, ku[0], kv[0]);
#pragma unroll
            for (int q = 0; q < 3; q++) {
                ku[0][q] *= ig0;
                kv[0][q] *= ig0;
            }
        }
        T stw = W0 * (ft * ig0), slen = W0 * ig0;
        bool ok = true;
        T b2min = b2;
#pragma unroll
        for (int st = 1; st < NS; st++) {
            T y[3];
#pragma unroll
            for (int q = 0; q < 3; q++) {
                T acc;
                if (SCH == SCH_RK4) {
                    acc = st == 3 ? k[2][q] : T(0.5) * k[st - 1][q];
                } else if (SCH == SCH_RK4_38) {
                    if (st == 1) acc = T(1.0 / 3.0) * k[0][q];
                    else if (st == 2) acc = k[1][q] - T(1.0 / 3.0) * k[0][q];
                    else acc = (k[0][q] - k[1][q]) + k[2][q];
                } else if (st == 1) acc = A10 * k[0][q];
                else if (st == 2) acc = N::fma_(A21, k[1][q], A20 * k[0][q]);
                else if (st == 3) acc = N::fma_(A32, k[2][q], N::fma_(A31, k[1][q], A30 * k[0][q]));
                else if (st == 4)
                    acc = N::fma_(A43, k[3][q],
                                  N::fma_(A42, k[2][q], N::fma_(A41, k[1][q], A40 * k[0][q])));
                else
                    acc = N::fma_(A54, k[4][q],
                                  N::fma_(A53, k[3][q],
                                          N::fma_(A52, k[2][q], N::fma_(A51, k[1][q], A50 * k[0][q]))));
                y[q] = N::fma_(H, acc, q == 0 ? L.p0 : (q == 1 ? L.p1 : L.p2));
            }
            T uy[3], vy[3];
            if constexpr (M2) {
#pragma unroll
                for (int q = 0; q < 3; q++) {
                    T au, av;
                    if (st == 1) au = A10 * ku[0][q], av = A10 * kv[0][q];
                    else if (st == 2) {
                        au = N::fma_(A21, ku[1][q], A20 * ku[0][q]);
                        av = N::fma_(A21, kv[1][q], A20 * kv[0][q]);
                    } else if (st == 3) {
                        au = N::fma_(A32, ku[2][q], N::fma_(A31, ku[1][q], A30 * ku[0][q]));
                        av = N::fma_(A32, kv[2][q], N::fma_(A31, kv[1][q], A30 * kv[0][q]));
                    } else if (st == 4) {
                        au = N::fma_(A43, ku[3][q], N::fma_(A42, ku[2][q], N::fma_(A41, ku[1][q], A40 * ku[0][q])));
                        av = N::fma_(A43, kv[3][q], N::fma_(A42, kv[2][q], N::fma_(A41, kv[1][q], A40 * kv[0][q])));
                    } else {
                        au = N::fma_(A54, ku[4][q], N::fma_(A53, ku[3][q],
                             N::fma_(A52, ku[2][q], N::fma_(A51, ku[1][q], A50 * ku[0][q]))));
                        av = N::fma_(A54, kv[4][q], N::fma_(A53, kv[3][q],
                             N::fma_(A52, kv[2][q], N::fma_(A51, kv[1][q], A50 * kv[0][q]))));
                    }
                    uy[q] = N::fma_(H, au, tn->u[q]);
                    vy[q] = N::fma_(H, av, tn->v[q]);
                }
            }
            T g0s, g1s, g2s, gts, b2s;
            // the twist integrand of Fehlberg's stage 1 has weight zero in the
            // fifth-order sum
            if (!FIXED && st == 1)
                rhs<T, false>(cb, cj, y[0], y[1], y[2], L.sgn, K.rx, K.ry, K.rz, K.twk, g0s, g1s, g2s,
                              gts, b2s);
            else
                rhs<T, TW>(cb, cj, y[0], y[1], y[2], L.sgn, K.rx, K.ry, K.rz, K.twk, g0s, g1s, g2s,
                           gts, b2s);
            b2min = mn(b2min, b2s);
            if (!finite_(b2s)) ok = false;
            T g = T(1);
            if (axis >= 0) {
                g = sel3(axis, g0s, g1s, g2s);
                // a fixed-step scheme has no error estimate to catch a landing whose
                // independent variable turns badly within the step (a line meeting
                // the face at a small angle): it approaches with shorter plain steps
                // until the face coordinate's rate changes by at most a tenth
                if (!(g * hs > N::gmin) || (FIXED && fabs(g - g0) > T(0.1) * fabs(g0))) {
                    ok = false;
                    g = g0;
                }
            }
            const T ig = N::rcp(g);
            k[st][0] = g0s * ig;
            k[st][1] = g1s * ig;
            k[st][2] = g2s * ig;
            if constexpr (M2) {
                const T bx = poly<T>(cb[0], y[0], y[1], y[2]), by = poly<T>(cb[1], y[0], y[1], y[2]),
                        bz = poly<T>(cb[2], y[0], y[1], y[2]);
                tan_rates<T>(cb, y[0], y[1], y[2], bx, by, bz, N::rsq(b2s), L.sgn, K.rx, K.ry, K.rz,
                             uy, vy, ku[st], kv[st]);
#pragma unroll
                for (int q = 0; q < 3; q++) {
                    ku[st][q] *= ig;
                    kv[st][q] *= ig;
                }
            }
            T bs;
            if (SCH == SCH_RK4) bs = st == 3 ? T(1.0 / 6.0) : T(1.0 / 3.0);
            else if (SCH == SCH_RK4_38) bs = st == 3 ? T(1.0 / 8.0) : T(3.0 / 8.0);
            else bs = st == 2 ? B2 : st == 3 ? B3 : st == 4 ? B4 : st == 5 ? B5 : T(0);
            if (FIXED || st != 1) stw = N::fma_(bs, gts * ig, stw);
            if (FIXED || st != 1) slen = N::fma_(bs, ig, slen);
        }
        T dyv[3], e[3];
#pragma unroll
        for (int q = 0; q < 3; q++) {
            if (SCH == SCH_RK4) {
                dyv[q] = H * (T(1.0 / 6.0) * (k[0][q] + k[3][q]) + T(1.0 / 3.0) * (k[1][q] + k[2][q]));
                e[q] = T(0);
            } else if (SCH == SCH_RK4_38) {
                dyv[q] = H * (T(1.0 / 8.0) * (k[0][q] + k[3][q]) + T(3.0 / 8.0) * (k[1][q] + k[2][q]));
                e[q] = T(0);
            } else {
                const T acc = N::fma_(B5, k[5][q], N::fma_(B4, k[4][q],
                              N::fma_(B3, k[3][q], N::fma_(B2, k[2][q], B0 * k[0][q]))));
                dyv[q] = H * acc;
                const T ea = N::fma_(E5, k[5][q], N::fma_(E4, k[4][q],
                             N::fma_(E3, k[3][q], N::fma_(E2, k[2][q], E0 * k[0][q]))));
                e[q] = H * ea;
            }
        }
        if (b2min <= K.bnull2) {
            fin_st = kNull;
            return;
        }
        T err2 = N::fma_(e[0], e[0], N::fma_(e[1], e[1], e[2] * e[2]));
        T du[3], dvv[3];
        if constexpr (M2) {
            // the tangent vectors' errors join the norm relative to their size (at
            // least one grid unit), as their 5th-order updates are formed
            T eu2 = T(0), ev2 = T(0);
#pragma unroll
            for (int q = 0; q < 3; q++) {
                du[q] = H * N::fma_(B5, ku[5][q], N::fma_(B4, ku[4][q],
                            N::fma_(B3, ku[3][q], N::fma_(B2, ku[2][q], B0 * ku[0][q]))));
                dvv[q] = H * N::fma_(B5, kv[5][q], N::fma_(B4, kv[4][q],
                             N::fma_(B3, kv[3][q], N::fma_(B2, kv[2][q], B0 * kv[0][q]))));
                const T a = H * N::fma_(E5, ku[5][q], N::fma_(E4, ku[4][q],
                                N::fma_(E3, ku[3][q], N::fma_(E2, ku[2][q], E0 * ku[0][q]))));
                const T b = H * N::fma_(E5, kv[5][q], N::fma_(E4, kv[4][q],
                                N::fma_(E3, kv[3][q], N::fma_(E2, kv[2][q], E0 * kv[0][q]))));
                eu2 = N::fma_(a, a, eu2);
                ev2 = N::fma_(b, b, ev2);
            }
            const T uu = mx(T(1), N::fma_(tn->u[0], tn->u[0], N::fma_(tn->u[1], tn->u[1], tn->u[2] * tn->u[2])));
            const T vv = mx(T(1), N::fma_(tn->v[0], tn->v[0], N::fma_(tn->v[1], tn->v[1], tn->v[2] * tn->v[2])));
            err2 = err2 + eu2 * N::rcp(uu) + ev2 * N::rcp(vv);
        }
        const T tol2 = L.tol * L.tol;
        const T s_step = H * ig0;  // arc length of the step, reference lengths
        if (!ok || !finite_(err2)) {
            if (axis < 0) {
                fin_st = kNonFinite;  // a NaN/Inf in the field
            } else {
                // the landing parametrisation broke down (the line turns within the
                // step): approach with shorter plain steps. Every failure shrinks h
                // below both the current h and the step just tried, so the plain-step
                // fallback always makes progress.
                L.h = mx(T(0.5) * mn(L.h, fabs(s_step)), N::hmin);
                ev(EV_LAND_BREAK);
            }
            return;
        }
        if (!FIXED && err2 > tol2) {  // reject: shrink and retry from the same point
            const float fac = fmaxf(0.9f * pow01((float)tol2 * Num<float>::rcp((float)err2)), 0.1f);
            L.h = mx((axis >= 0 ? mn(L.h, fabs(s_step)) : L.h) * (T)fac, N::hmin);
            ev(axis >= 0 ? EV_REJECT_LAND : EV_REJECT_ARC);
            return;
        }
        const float grow = err2 > T(0) ? fminf(0.9f * pow01((float)tol2 * Num<float>::rcp((float)err2)), 5.0f)
                                       : 5.0f;
        T n0 = L.p0 + dyv[0], n1 = L.p1 + dyv[1], n2 = L.p2 + dyv[2];
        const T ov = M2 ? N::ov_tan : N::ov;
        // Past a box face the line ends on that face, and clamping an overshoot d onto
        // it moves the end by d over the line's slope to the face: a first-order
        // error, not the second-order kink error of an interior face. So a step that
        // ends past a box face the line crosses keeps no overshoot: it lands on that
        // face instead (`bp`, its face code), or, where the line is not heading out
        // steeply enough at the step's start to take the face coordinate as the
        // independent variable, approaches it with shorter plain steps first. Only
        // a line tangent to the box face at both ends of the step keeps the
        // allowance. The start direction is k1 times g0; stage 5 sits at the end
        // of the step, so k5 times g0 stands for the end direction (its sign is
        // exact, its size is scaled by that stage's own g on a landing).
        constexpr int KE = FIXED ? 3 : 4;  // the stage at the end of the step (c = 1)
        int bp = -1;
        if (axis != 0) bp = box_past(n0, L.c0, K.nx, k[0][0] * g0, k[KE][0] * g0, 0);
        if (bp < 0 && axis != 1) bp = box_past(n1, L.c1, K.ny, k[0][1] * g0, k[KE][1] * g0, 2);
        if (bp < 0 && axis != 2) bp = box_past(n2, L.c2, K.nz, k[0][2] * g0, k[KE][2] * g0, 4);
        // a brief excursion over a face inside the step (the end may be back inside)
        int xf = -1;
        if (axis != 0) xf = excursion(0, L.p0, H * k[0][0], dyv[0], ov);
        if (xf < 0 && axis != 1) xf = excursion(1, L.p1, H * k[0][1], dyv[1], ov);
        if (xf < 0 && axis != 2) xf = excursion(2, L.p2, H * k[0][2], dyv[2], ov);
        if (axis < 0) {
            if (xf < 0 && bp < 0 && n0 >= -ov && n0 <= T(1) + ov && n1 >= -ov && n1 <= T(1) + ov &&
                n2 >= -ov && n2 <= T(1) + ov) {
                // inside, or past a face by at most ov: a step straddling a face by d
                // errs by O(d^2), so keep it and carry the overshoot into the
                // neighbouring cell (on a box face, clamp to it)
                L.p0 = n0;
                L.p1 = n1;
                L.p2 = n2;
                if constexpr (M2)
#pragma unroll
                    for (int q = 0; q < 3; q++) {
                        tn->u[q] += du[q];
                        tn->v[q] += dvv[q];
                    }
                int cl = 0;
                bool moved = carry(L.c0, L.p0, K.nx, cl, 1);
                moved |= carry(L.c1, L.p1, K.ny, cl, 2);
                moved |= carry(L.c2, L.p2, K.nz, cl, 4);
                if (moved) need_load = true;
                L.tw += (double)(H * stw);
                L.len += (double)(H * slen);
                L.h = FIXED ? L.tol : mn(L.h * (T)grow, T(4));
                n_acc++;
                ev.accepted(-1, H, cl);
                ev(EV_ACCEPT_ARC);
            } else {
                // the line curved out of the cell before the straight-line guess: land
                // next on the face its chord crossed first
                T th = T(2), tq;
                int fb = -1;
                if (n0 > T(1)) { tq = (T(1) - L.p0) / (n0 - L.p0); if (tq < th) th = tq, fb = 1; }
                else if (n0 < T(0)) { tq = -L.p0 / (n0 - L.p0); if (tq < th) th = tq, fb = 0; }
                if (n1 > T(1)) { tq = (T(1) - L.p1) / (n1 - L.p1); if (tq < th) th = tq, fb = 3; }
                else if (n1 < T(0)) { tq = -L.p1 / (n1 - L.p1); if (tq < th) th = tq, fb = 2; }
                if (n2 > T(1)) { tq = (T(1) - L.p2) / (n2 - L.p2); if (tq < th) th = tq, fb = 5; }
                else if (n2 < T(0)) { tq = -L.p2 / (n2 - L.p2); if (tq < th) th = tq, fb = 4; }
                if (fb < 0) fb = xf, th = T(0.5);
                L.force = fb;
                L.h = mx(L.h * mn(mx(th, T(0.5)), T(1)), N::hmin);
                ev(EV_CURVED_OUT);
            }
            return;
        }
        // landing step: the other coordinates must still be within ov of the cell, and
        // not past a box face the line heads out through
        int fb = bp >= 0 ? bp : xf;
        if (axis != 0 && (n0 < -ov || n0 > T(1) + ov)) fb = n0 > T(1) ? 1 : 0;
        if (axis != 1 && (n1 < -ov || n1 > T(1) + ov)) fb = n1 > T(1) ? 3 : 2;
        if (axis != 2 && (n2 < -ov || n2 > T(1) + ov)) fb = n2 > T(1) ? 5 : 4;
        if (fb >= 0) {
            // another face comes first: land there next, unless this already was a
            // forced landing (then approach with plain steps, which always progress)
            if (want == 0) L.force = fb;
            L.h = mx(T(0.5) * mn(L.h, fabs(s_step)), N::hmin);
            ev(EV_LAND_OTHER);
            return;
        }
        const int d = hs > 0 ? 1 : -1;
        if constexpr (M2)
#pragma unroll
            for (int q = 0; q < 3; q++) {
                tn->u[q] += du[q];
                tn->v[q] += dvv[q];
            }
        L.p0 = axis == 0 ? (d > 0 ? T(1) : T(0)) : n0;
        L.p1 = axis == 1 ? (d > 0 ? T(1) : T(0)) : n1;
        L.p2 = axis == 2 ? (d > 0 ? T(1) : T(0)) : n2;
        L.tw += (double)(H * stw);
        L.len += (double)(H * slen);
        // a landing is cut short by the face, not by the error bound: unless the error
        // asks for a smaller step, keep the step the controller had before the cut
        if (FIXED) L.h = L.tol;
        else L.h = grow >= 1.0f ? mn(mx(fabs(s_step) * (T)grow, L.h), T(4)) : fabs(s_step) * (T)grow;
        n_acc++;
        // carry small overshoots of the other coordinates (a crossing near an edge)
        bool moved = false;
        int cl = 0;
        if (axis != 0) moved |= carry(L.c0, L.p0, K.nx, cl, 1);
        if (axis != 1) moved |= carry(L.c1, L.p1, K.ny, cl, 2);
        if (axis != 2) moved |= carry(L.c2, L.p2, K.nz, cl, 4);
        if (moved) need_load = true;
        ev.accepted(axis, H, cl);
        ev(EV_ACCEPT_LAND);
        xa = axis;
        xd = d;
    }
    // cross face xa in direction xd: the next cell, or the end of the line
    if (xa < 0) return;
    if (xa == 0) {
        if (xd > 0) { if (L.c0 == K.nx - 2) fin_st = 0, fin_face = 1; else L.c0++, L.p0 = T(0); }
        else { if (L.c0 == 0) fin_st = 0, fin_face = 0; else L.c0--, L.p0 = T(1); }
    } else if (xa == 1) {
        if (xd > 0) { if (L.c1 == K.ny - 2) fin_st = 0, fin_face = 3; else L.c1++, L.p1 = T(0); }
        else { if (L.c1 == 0) fin_st = 0, fin_face = 2; else L.c1--, L.p1 = T(1); }
    } else {
        if (xd > 0) { if (L.c2 == K.nz - 2) fin_st = 0, fin_face = 5; else L.c2++, L.p2 = T(0); }
        else { if (L.c2 == 0) fin_st = 0, fin_face = 4; else L.c2--, L.p2 = T(1); }
    }
    if (fin_st < 0) need_load = true;
}

}  // namespace fq
