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
