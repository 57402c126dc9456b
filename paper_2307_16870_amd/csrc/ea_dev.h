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
// formed in FP64 whatever the working type: formed in FP32 their rounding
// leaves the accumulated rotation slightly non-unitary on average, which
// over the ~n * sweeps rotations a column receives shows up as a drift of the
// column norms (the singular values) of order 1e-5 at n = 2048.  Returns
// false when the pair is already orthogonal to tolerance.
template <typename T>
struct JRot {
    T s, gm, tg;  // sin, 1 - cos, t * |ga|
    cx<T> e;
};
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

// One rotation of a Jacobi step as staged in LDS for the update threads.
template <typename T>
struct alignas(16) RotRec {
    T s, gm;   // sin, 1 - cos
    cx<T> e;   // phase conj(g) / |g|
    T tg;      // t |g|
    T al, be;  // diagonal entries before the rotation
    int on;    // rotation applied
};
