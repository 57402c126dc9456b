// Device-side complex arithmetic and launch helpers shared by the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T x, y;
};

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T a, T b) { cx<T> r; r.x = a; r.y = b; return r; }
template <typename T>
__device__ __forceinline__ cx<T> zero_cx() { return mk<T>(T(0), T(0)); }
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return mk<T>(s * a.x, s * a.y); }
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return mk<T>(a.x, -a.y); }
// acc += a * b
template <typename T>
__device__ __forceinline__ void cmac(cx<T> &acc, cx<T> a, cx<T> b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
template <typename T>
__device__ __forceinline__ void cmacc(cx<T> &acc, cx<T> a, cx<T> b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
}
template <typename T>
__device__ __forceinline__ T norm2(cx<T> a) { return a.x * a.x + a.y * a.y; }

// Round-robin ("circle method") tournament: player in `slot` at round `rnd`
// over n_even players.  Slot i plays slot n_even-1-i.
__device__ __forceinline__ int rr_player(int slot, int rnd, int n_even) {
    if (slot == 0) return 0;
    return (slot - 1 + rnd) % (n_even - 1) + 1;
}

// Plane rotation [op, oq] = [xp, yq] [[c, s], [-s, c]] with c = sqrt(1 - s^2)
// entering only through gm = s^2 / (1 + c) = 1 - c.  Written as a correction
// to the identity so that a rotation with t^2 below the unit roundoff (where c
// itself rounds to 1) still keeps c^2 + s^2 = 1 to working precision instead
// of inflating both columns by 1 + t^2; summed over the many small rotations
// of the last sweeps that bias would otherwise grow the column norms of an
// FP32 factorisation by O(1e-3) at n = 2048.
template <typename T>
__device__ __forceinline__ void rot_pair(cx<T> xp, cx<T> yq, T s, T gm, cx<T> &op, cx<T> &oq) {
    op = xp - (gm * xp + s * yq);
    oq = yq + (s * xp - gm * yq);
}

// Rotation that zeroes the off-diagonal entry of the Hermitian 2x2 block
// [[al, ga], [conj(ga), be]] of a Gram matrix (one-sided Jacobi, Hestenes):
// tan(theta) = t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
// zeta = (be - al) / (2 |ga|), phase e = conj(ga) / |ga|.  The parameters are
// formed in FP64 whatever the working type: with FP32 working data, angles
// formed in FP32 (one-ulp reciprocal square roots) were measured to raise the
// end-to-end error of a 490-update circuit tenfold.  Returns false when the
// pair is already orthogonal to tolerance.
template <typename T>
struct JRot {
    T s, gm, tg;  // sin, 1 - cos, t * |ga|
    cx<T> e;
};
// FP64 reciprocal square root and reciprocal from the hardware estimates
// refined by two Newton steps each (y <- y (3 - x y^2) / 2, y <- y (2 - x y));
// arguments are positive and finite here.  Far fewer dependent instructions
// than the correctly rounded division and square root, to about one ulp.
__device__ __forceinline__ double rsq_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * fma(-hx * y, y, 1.5);
    y = y * fma(-hx * y, y, 1.5);
    return y;
}
__device__ __forceinline__ double rcp_nr(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = y * fma(-x, y, 2.0);
    y = y * fma(-x, y, 2.0);
    return y;
}
template <typename T>
__device__ __forceinline__ bool jacobi_rotation(T al_, T be_, cx<T> ga_, T tol, JRot<T> &r) {
    const double al = al_, be = be_, gx = ga_.x, gy = ga_.y;
    const double g = sqrt(gx * gx + gy * gy);
    if (!(g > 0.0) || !(g > (double)tol * sqrt(al * be))) return false;
    const double zeta = (be - al) / (2.0 * g), az = fabs(zeta);
    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (az + (az < 1e150 ? sqrt(1.0 + az * az) : az));
    const double c = 1.0 / sqrt(1.0 + t * t), s = c * t, ig = 1.0 / g;
    r.s = (T)s;
    r.gm = (T)(s * s / (1.0 + c));
    r.tg = (T)(t * g);
    r.e = mk<T>((T)(gx * ig), (T)(-gy * ig));
    return true;
}
// FP32 working data: the same FP64 formulas with Newton-refined reciprocals
// (their one-sided error of a fraction of an FP64 ulp is far below FP32
// rounding, while the correctly rounded FP64 forms lengthen the critical path
// of every Jacobi step).
template <>
__device__ __forceinline__ bool jacobi_rotation<float>(float al_, float be_, cx<float> ga_,
                                                       float tol, JRot<float> &r) {
    const double al = al_, be = be_, gx = ga_.x, gy = ga_.y;
    const double g2 = gx * gx + gy * gy, ab = al * be;
    if (!(g2 > 0.0)) return false;
    const double ig = rsq_nr(g2), g = g2 * ig;
    // g > tol sqrt(al be); a negative product (rounding of a vanishing
    // column) never rotates, as sqrt would give NaN
    if (!(ab >= 0.0) || !(g > (double)tol * (ab > 0.0 ? ab * rsq_nr(ab) : 0.0))) return false;
    const double zeta = (be - al) * 0.5 * ig, az = fabs(zeta);
    const double h = 1.0 + az * az;
    const double t = (zeta >= 0.0 ? 1.0 : -1.0) * rcp_nr(az + (az < 1e150 ? h * rsq_nr(h) : az));
    const double c = rsq_nr(1.0 + t * t), s = c * t;
    r.s = (float)s;
    r.gm = (float)(s * s * rcp_nr(1.0 + c));
    r.tg = (float)(t * g);
    r.e = mk<float>((float)(gx * ig), (float)(-gy * ig));
    return true;
}

// One rotation of a Jacobi step as staged in LDS for the update threads.
template <typename T>
struct alignas(16) RotRec {
    T s, gm;   // sin, 1 - cos
    cx<T> e;   // phase conj(g) / |g|
    T tg;      // t |g|
    T al, be;  // diagonal entries before the rotation
    int on;    // rotation applied
};
