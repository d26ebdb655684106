// Interleaved complex type used by the kernels (FP64 or FP32 parts).
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace mb {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T x, y;
};

template <typename T>
__host__ __device__ inline cx<T> mk(T a, T b) {
    cx<T> r;
    r.x = a;
    r.y = b;
    return r;
}
template <typename T>
__device__ inline cx<T> cadd(cx<T> a, cx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ inline cx<T> csub(cx<T> a, cx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ inline cx<T> cmul(cx<T> a, cx<T> b) {
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <typename T>
__device__ inline cx<T> cmulc(cx<T> a, cx<T> b) {
    return mk<T>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
template <typename T>
__device__ inline cx<T> cscale(cx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
// acc += a * b
template <typename T>
__device__ inline void cfma(cx<T>& acc, cx<T> a, cx<T> b) {
    acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
    acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}
// acc += conj(a) * b
template <typename T>
__device__ inline void cfmac(cx<T>& acc, cx<T> a, cx<T> b) {
    acc.x = fma(a.x, b.x, fma(a.y, b.y, acc.x));
    acc.y = fma(a.x, b.y, fma(-a.y, b.x, acc.y));
}

// Map a flat block index so that consecutive logical indices land on the same
// XCD: hardware assigns block b to XCD (b mod 8); logical order runs through all
// blocks of XCD 0 first, then XCD 1, ...  Valid for any grid size.
__device__ inline unsigned xcd_logical(unsigned b, unsigned nblocks) {
    const unsigned nx = 8;
    unsigned x = b % nx, k = b / nx;
    unsigned base = nblocks / nx, rem = nblocks % nx;
    // XCD x owns base + (x < rem) blocks; logical start of XCD x
    unsigned start = x * base + (x < rem ? x : rem);
    return start + k;
}

// Work units of a batch: item t owns units [unit_begin[t], unit_begin[t+1]);
// returns the item that owns unit u (unit_begin ascending, unit_begin[0] = 0).
__device__ inline int batch_item_of(const int32_t* unit_begin, int n, unsigned u) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if ((unsigned)unit_begin[mid] <= u) lo = mid; else hi = mid - 1;
    }
    return lo;
}

}  // namespace mb
