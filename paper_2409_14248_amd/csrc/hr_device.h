// hr_device.h -- device-side building blocks shared by the HRKAN kernels:
// grid parameters, the HR basis with its first three derivatives, and the
// jet-channel bookkeeping.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hrk {

// Uniform grid of G intervals on [lo, hi]; basis b lives on
// [lo + (b-k) h, lo + (b+1) h] (the order-k B-spline supports, Sec. 2.1-2.2).
// Kernels work in the scaled coordinate zeta = (z - lo) * inv_w, in which
// every support has width 2 and the knots sit at multiples of kappa =
// 2/(k+1) (0.5 for k = 3: exact in binary, so no knot-position rounding).
template <typename T>
struct GridP {
    T lo;         // grid start
    T inv_w;      // 2 / ((k+1) h)
    T kappa;      // 2 / (k+1): one grid interval in zeta units
    T inv_kappa;  // (k+1) / 2
    int k;        // supports span k+1 intervals
    int nb;       // G + k basis functions
    int m;        // HR order
};

// Jet channels of a layer's features, fixed at compile time by the order of
// differentiation along the two input coordinates: O0 along x0 and O1 along
// x1 (0..5 each). Channel order: U, the x0-derivatives of order 1..O0, the
// x1-derivatives of order 1..O1; for orders up to two U, X, XX, Y, YY
// (absent ones skipped).
template <int O0, int O1>
struct Ch {
    static constexpr int C = 1 + O0 + O1;
    static constexpr int OM = O0 > O1 ? O0 : O1;      // highest order
    static constexpr bool LOW = O0 <= 2 && O1 <= 2;    // at most second order
    static constexpr int U = 0;
    static constexpr int X = O0 >= 1 ? 1 : -1;
    static constexpr int XX = O0 >= 2 ? 2 : -1;
    static constexpr int Y = O1 >= 1 ? 1 + O0 : -1;
    static constexpr int YY = O1 >= 2 ? 2 + O0 : -1;
    // channel of the k-th derivative (k >= 1) along x0 / x1
    static constexpr int xk(int k) { return k; }
    static constexpr int yk(int k) { return O0 + k; }
};

template <typename T>
__device__ __forceinline__ T ipow(T v, int e)
{
    T r = T(1);
    for (int i = 0; i < e; ++i) r *= v;
    return r;
}

template <typename T>
__device__ __forceinline__ T zeta_of(const GridP<T> &g, T z)
{
    return (z - g.lo) * g.inv_w;
}

// Interval index floor(zeta / kappa) = floor((z - lo) / h), clamped so that
// far-away or infinite z give an index whose k+1 candidate bumps are all
// outside 0..nb-1 (a zero basis); NaN maps to 0 so that the bumps evaluated
// there carry the NaN.
template <typename T>
__device__ __forceinline__ int interval_of(const GridP<T> &g, T zeta)
{
    T u = zeta * g.inv_kappa;
    const T lim = T(g.nb + 2);
    if (!(u == u)) return 0;
    u = u < -lim ? -lim : (u > lim ? lim : u);
    return (int)floor(u);
}

// HR bump b of order m at scaled coordinate zeta, and its z-derivatives up
// to ND (2 or 3). With a = zeta - (b-k) kappa and be = (b+1) kappa - zeta
// (both in [0, 2] inside the support), t = a * be and d = be - a:
//   v    = t^m
//   v'   = inv_w   * m * t^(m-1) * d
//   v''  = inv_w^2 * m * t^(m-2) * ((m-1) d^2 - 2 t)
//   v''' = inv_w^3 * m (m-1) * t^(m-3) * d * ((m-2) d^2 - 6 t)     (m >= 3)
//        = -12 * inv_w^3 * d                                      (m == 2)
// This is c_m (e-z)^m (z-s)^m of Eq. 2 differentiated through t(z), written in
// the scaled variables; zero outside the open support.
// MC > 0 fixes the order at compile time (no power loops); MC = 0 reads it
// from the grid.
template <typename T, int ND, int MC = 0>
__device__ __forceinline__ void hr_bump(const GridP<T> &g, T zeta, int b, T *v)
{
    const T a = zeta - T(b - g.k) * g.kappa;
    const T be = T(b + 1) * g.kappa - zeta;
    const bool in = (a > T(0)) && (be > T(0)) && b >= 0 && b < g.nb;
    const T t = a * be;
    const T d = be - a;
    const int m = MC > 0 ? MC : g.m;
    const T tm2 = ipow(t, m - 2);
    const T fm = T(m);
    T v0 = tm2 * t * t;
    T v1 = g.inv_w * fm * tm2 * t * d;
    T v2 = g.inv_w * g.inv_w * fm * tm2 * (T(m - 1) * d * d - T(2) * t);
    v[0] = in ? v0 : T(0);
    v[1] = in ? v1 : T(0);
    v[2] = in ? v2 : T(0);
    if constexpr (ND >= 3) {
        const T w3 = g.inv_w * g.inv_w * g.inv_w;
        T v3;
        if (m == 2)
            v3 = T(-12) * w3 * d;
        else
            v3 = w3 * fm * T(m - 1) * ipow(t, m - 3) * d * (T(m - 2) * d * d - T(6) * t);
        v[3] = in ? v3 : T(0);
    }
    if (!(zeta == zeta)) {                  // propagate NaN inputs
        v[0] = zeta; v[1] = zeta; v[2] = zeta;
        if constexpr (ND >= 3) v[3] = zeta;
    }
}

// HR bump b and its z-derivatives of order 0..ND (ND up to 8) at scaled
// coordinate zeta. With t = a be and d = be - a as above, t' = d and
// t'' = -2 in zeta, so (Faa di Bruno for an inner function of degree two)
//   d^j t^m / dzeta^j = sum_{i=0}^{j/2} j! / (i! (j-2i)!) (-1)^i d^(j-2i)
//                       * m! / (m-j+i)! * t^(m-j+i),
// terms with j - i > m being zero; each zeta-derivative is then scaled by
// inv_w^j. Zero outside the open support; NaN zeta propagates.
template <typename T, int ND>
__device__ __forceinline__ void hr_bump_n(const GridP<T> &g, T zeta, int b, T *v)
{
    const T a = zeta - T(b - g.k) * g.kappa;
    const T be = T(b + 1) * g.kappa - zeta;
    const bool in = (a > T(0)) && (be > T(0)) && b >= 0 && b < g.nb;
    const T t = a * be;
    const T d = be - a;
    const int m = g.m;
    // powers d^0..d^ND
    T dp[ND + 1];
    dp[0] = T(1);
#pragma unroll
    for (int e = 1; e <= ND; ++e) dp[e] = dp[e - 1] * d;
    T sc = T(1);
#pragma unroll
    for (int j = 0; j <= ND; ++j) {
        T sum = T(0);
        T jf = T(1);                                  // j! / (i! (j-2i)!) by recurrence in i
#pragma unroll
        for (int i = 0; 2 * i <= j; ++i) {
            const int r = j - i;                      // order of the derivative of t^m
            if (i > 0) jf = jf * T((j - 2 * i + 2) * (j - 2 * i + 1)) / T(i);
            if (r <= m) {
                T fall = T(1);                        // m! / (m-r)!
                for (int q = 0; q < r; ++q) fall *= T(m - q);
                const T term = jf * dp[j - 2 * i] * fall * ipow(t, m - r);
                sum += (i & 1) ? -term : term;
            }
        }
        v[j] = in ? sum * sc : T(0);
        sc *= g.inv_w;
    }
    if (!(zeta == zeta))
#pragma unroll
        for (int j = 0; j <= ND; ++j) v[j] = zeta;
}

// Jets of any order along one coordinate through one basis function, in
// normalised Taylor coefficients: with c_i = z^(i) / i! (i = 1..N) and
// delta(h) = sum_i c_i h^i, v(z0 + delta) = sum_j v^(j) / j! delta^j, so the
// k-th derivative of the feature is k! sum_{j=1..k} v^(j) / j! [h^k] delta^j.
// P[j][k] = [h^k] delta^j, built by repeated truncated products.
template <typename T, int N>
__device__ __forceinline__ void taylor_powers(const T *c, T (*P)[N + 1])
{
#pragma unroll
    for (int k = 0; k <= N; ++k) P[0][k] = k == 0 ? T(1) : T(0);
#pragma unroll
    for (int j = 1; j <= N; ++j)
#pragma unroll
        for (int k = 0; k <= N; ++k) {
            T s = T(0);
#pragma unroll
            for (int i = 1; i <= k; ++i) s += c[i] * P[j - 1][k - i];
            P[j][k] = s;
        }
}

__device__ __forceinline__ constexpr double fact_d(int n) { return n <= 1 ? 1.0 : n * fact_d(n - 1); }

// Features of one coordinate's channels: A[k-1] = d^k/dx^k v(z(x)), k = 1..N,
// from the derivatives zd[1..N] of z and v[0..N] of the bump.
template <typename T, int N>
__device__ __forceinline__ void taylor_features(const T *v, const T *zd, T *A)
{
    T c[N + 1];
    c[0] = T(0);
#pragma unroll
    for (int i = 1; i <= N; ++i) c[i] = zd[i] * T(1.0 / fact_d(i));
    T P[N + 1][N + 1];
    taylor_powers<T, N>(c, P);
#pragma unroll
    for (int k = 1; k <= N; ++k) {
        T s = T(0);
#pragma unroll
        for (int j = 1; j <= k; ++j) s += v[j] * T(1.0 / fact_d(j)) * P[j][k];
        A[k - 1] = s * T(fact_d(k));
    }
}

// Reverse of taylor_features: add to *z0b the bar of z (through v^(j+1))
// and to zdb[i] the bars of z^(i), given the feature bars Ab[k-1]:
//   dA_k/dz     = k! sum_j v^(j+1) / j! P[j][k],
//   dA_k/dz^(i) = k! / i! sum_j v^(j) / (j-1)! P[j-1][k-i]   (d[h^k]delta^j/dc_i = j [h^(k-i)]delta^(j-1)).
template <typename T, int N>
__device__ __forceinline__ void taylor_adjoint(const T *v, const T *zd, const T *Ab, T *z0b, T *zdb)
{
    T c[N + 1];
    c[0] = T(0);
#pragma unroll
    for (int i = 1; i <= N; ++i) c[i] = zd[i] * T(1.0 / fact_d(i));
    T P[N + 1][N + 1];
    taylor_powers<T, N>(c, P);
#pragma unroll
    for (int k = 1; k <= N; ++k) {
        const T ab = Ab[k - 1] * T(fact_d(k));
        T dz = T(0);
#pragma unroll
        for (int j = 1; j <= k; ++j) dz += v[j + 1] * T(1.0 / fact_d(j)) * P[j][k];
        *z0b += ab * dz;
#pragma unroll
        for (int i = 1; i <= k; ++i) {
            T di = T(0);
#pragma unroll
            for (int j = 1; j <= k - i + 1; ++j) di += v[j] * T(1.0 / fact_d(j - 1)) * P[j - 1][k - i];
            zdb[i] += ab * T(1.0 / fact_d(i)) * di;
        }
    }
}

// Features of one basis function for one point, per channel:
//   A_U = v, A_X = v' zx, A_XX = v'' zx^2 + v' zxx, A_Y = v' zy, A_YY = v'' zy^2 + v' zyy
template <typename T, int O0, int O1>
__device__ __forceinline__ void features(const T *v, const T *zj, T *A)
{
    using CH = Ch<O0, O1>;
    if constexpr (!CH::LOW) {
        // any order: v[0..OM] (hr_bump_n), per coordinate in Taylor form
        A[CH::U] = v[0];
        if constexpr (O0 > 0) {
            T zd[O0 + 1];
            zd[0] = T(0);
#pragma unroll
            for (int k = 1; k <= O0; ++k) zd[k] = zj[CH::xk(k)];
            taylor_features<T, O0>(v, zd, A + CH::xk(1));
        }
        if constexpr (O1 > 0) {
            T zd[O1 + 1];
            zd[0] = T(0);
#pragma unroll
            for (int k = 1; k <= O1; ++k) zd[k] = zj[CH::yk(k)];
            taylor_features<T, O1>(v, zd, A + CH::yk(1));
        }
        return;
    }
    A[CH::U] = v[0];
    if constexpr (CH::X >= 0) A[CH::X] = v[1] * zj[CH::X];
    if constexpr (CH::XX >= 0) A[CH::XX] = v[2] * zj[CH::X] * zj[CH::X] + v[1] * zj[CH::XX];
    if constexpr (CH::Y >= 0) A[CH::Y] = v[1] * zj[CH::Y];
    if constexpr (CH::YY >= 0) A[CH::YY] = v[2] * zj[CH::Y] * zj[CH::Y] + v[1] * zj[CH::YY];
}

// Reverse of `features`: add d(sum_c Ab_c A_c)/d(jets) to zb, given the bars
// Ab of the features and the basis derivatives v (up to v''').
template <typename T, int O0, int O1>
__device__ __forceinline__ void features_adjoint(const T *v, const T *zj, const T *Ab, T *zb)
{
    using CH = Ch<O0, O1>;
    if constexpr (!CH::LOW) {
        // any order: v[0..OM+1] (hr_bump_n)
        T z0 = Ab[CH::U] * v[1];
        if constexpr (O0 > 0) {
            T zd[O0 + 1], zdb[O0 + 1];
#pragma unroll
            for (int k = 0; k <= O0; ++k) {
                zd[k] = k == 0 ? T(0) : zj[CH::xk(k)];
                zdb[k] = T(0);
            }
            taylor_adjoint<T, O0>(v, zd, Ab + CH::xk(1), &z0, zdb);
#pragma unroll
            for (int k = 1; k <= O0; ++k) zb[CH::xk(k)] += zdb[k];
        }
        if constexpr (O1 > 0) {
            T zd[O1 + 1], zdb[O1 + 1];
#pragma unroll
            for (int k = 0; k <= O1; ++k) {
                zd[k] = k == 0 ? T(0) : zj[CH::yk(k)];
                zdb[k] = T(0);
            }
            taylor_adjoint<T, O1>(v, zd, Ab + CH::yk(1), &z0, zdb);
#pragma unroll
            for (int k = 1; k <= O1; ++k) zb[CH::yk(k)] += zdb[k];
        }
        zb[CH::U] += z0;
        return;
    }
    T z0 = Ab[CH::U] * v[1];
    if constexpr (CH::X >= 0) {
        z0 += Ab[CH::X] * v[2] * zj[CH::X];
        zb[CH::X] += Ab[CH::X] * v[1];
    }
    if constexpr (CH::XX >= 0) {
        z0 += Ab[CH::XX] * (v[3] * zj[CH::X] * zj[CH::X] + v[2] * zj[CH::XX]);
        zb[CH::X] += Ab[CH::XX] * T(2) * v[2] * zj[CH::X];
        zb[CH::XX] += Ab[CH::XX] * v[1];
    }
    if constexpr (CH::Y >= 0) {
        z0 += Ab[CH::Y] * v[2] * zj[CH::Y];
        zb[CH::Y] += Ab[CH::Y] * v[1];
    }
    if constexpr (CH::YY >= 0) {
        z0 += Ab[CH::YY] * (v[3] * zj[CH::Y] * zj[CH::Y] + v[2] * zj[CH::YY]);
        zb[CH::Y] += Ab[CH::YY] * T(2) * v[2] * zj[CH::Y];
        zb[CH::YY] += Ab[CH::YY] * v[1];
    }
    zb[CH::U] += z0;
}

// Jets of input feature i (0 or 1) of layer 0 at point x: the coordinate
// itself with a unit first derivative along its own direction.
template <typename T, int O0, int O1>
__device__ __forceinline__ void input_jets(const T *x, int64_t p, int i, T *zj)
{
    using CH = Ch<O0, O1>;
    if constexpr (!CH::LOW) {
#pragma unroll
        for (int c = 0; c < CH::C; ++c) zj[c] = T(0);
        zj[CH::U] = x[2 * p + i];
        if constexpr (O0 > 0) zj[CH::xk(1)] = i == 0 ? T(1) : T(0);
        if constexpr (O1 > 0) zj[CH::yk(1)] = i == 1 ? T(1) : T(0);
        return;
    }
    zj[CH::U] = x[2 * p + i];
    if constexpr (CH::X >= 0) zj[CH::X] = i == 0 ? T(1) : T(0);
    if constexpr (CH::XX >= 0) zj[CH::XX] = T(0);
    if constexpr (CH::Y >= 0) zj[CH::Y] = i == 1 ? T(1) : T(0);
    if constexpr (CH::YY >= 0) zj[CH::YY] = T(0);
}

}  // namespace hrk
