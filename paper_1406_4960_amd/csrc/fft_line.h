// Small in-register FFTs with compile-time plans, shared by the fused local kernels.
//   line_fft<T, N, SIGN>(v): v[k] <- sum_j v[j] exp(SIGN 2 pi i j k / N), N a product of
//   2, 3, 4 and 5, as a mixed-radix Stockham sequence of radix stages held in registers.
// Twiddle factors are compile-time constants (kRoots<N>): after unrolling every one is an
// immediate operand.
#pragma once

#include "cplx.h"

namespace mb {
namespace fftl {

struct RadixPlan {
    int nr;
    int rad[12];
};

constexpr RadixPlan make_plan(int n) {
    RadixPlan p{0, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}};
    const int order[4] = {4, 2, 3, 5};
    for (int k = 0; k < 4; ++k)
        while (n % order[k] == 0) {
            p.rad[p.nr++] = order[k];
            n /= order[k];
        }
    return p;
}

template <int N>
struct LinePlan {
    static constexpr RadixPlan p = make_plan(N);
};

// Roots of unity exp(2 pi i m / N) as compile-time constants: the angle is reduced
// to an octant with integer arithmetic and sin / cos of the remaining |x| <= pi/4
// come from their Taylor series, nested from the smallest term (within 1e-16 of
// the exact values).  After unrolling every twiddle factor is an immediate operand.
struct SinCos {
    double s, c;
};

constexpr SinCos taylor_sincos(double x) {
    const double x2 = x * x;
    double s = 1.0, c = 1.0;
    for (int k = 13; k >= 1; --k) {
        s = 1.0 - s * x2 / ((2.0 * k) * (2.0 * k + 1.0));
        c = 1.0 - c * x2 / ((2.0 * k - 1.0) * (2.0 * k));
    }
    return SinCos{x * s, c};
}

constexpr SinCos unit_root(int m, int n) {
    m %= n;
    if (m < 0) m += n;
    const int o = (8 * m) / n;  // octant of the angle 2 pi m / n
    const double h = 2.0 * 3.14159265358979323846 / (8.0 * n);
    const SinCos a = taylor_sincos(h * (double)(8 * m - o * n));        // angle - o pi / 4
    const SinCos b = taylor_sincos(h * (double)((o + 1) * n - 8 * m));  // (o + 1) pi / 4 - angle
    switch (o) {
        case 0: return SinCos{a.s, a.c};
        case 1: return SinCos{b.c, b.s};
        case 2: return SinCos{a.c, -a.s};
        case 3: return SinCos{b.s, -b.c};
        case 4: return SinCos{-a.s, -a.c};
        case 5: return SinCos{-b.c, -b.s};
        case 6: return SinCos{-a.c, a.s};
        default: return SinCos{-b.s, b.c};
    }
}

template <int N>
struct RootTable {
    double c[N], s[N];
    constexpr RootTable() : c(), s() {
        for (int m = 0; m < N; ++m) {
            const SinCos v = unit_root(m, N);
            c[m] = v.c;
            s[m] = v.s;
        }
    }
};

template <int N>
__device__ constexpr RootTable<N> kRoots{};

// y_k = sum_r v_r exp(sign 2 pi i r k / R), R in {2, 3, 4, 5}
template <typename T, int R, int SIGN>
__device__ __forceinline__ void bfly(cx<T>* v) {
    constexpr T s = (T)SIGN;
    if constexpr (R == 2) {
        cx<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 4) {
        cx<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        cx<T> t2 = cadd(v[1], v[3]), d = csub(v[1], v[3]);
        cx<T> t3 = mk<T>(-s * d.y, s * d.x);
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    } else if constexpr (R == 3) {
        const T c3 = (T)-0.5;
        const T s3 = (T)0.86602540378443864676;
        cx<T> t = cadd(v[1], v[2]), d = csub(v[1], v[2]);
        cx<T> a = mk<T>(v[0].x + c3 * t.x, v[0].y + c3 * t.y);
        const T ss = s * s3;
        cx<T> b = mk<T>(-ss * d.y, ss * d.x);
        v[0] = cadd(v[0], t);
        v[1] = cadd(a, b);
        v[2] = csub(a, b);
    } else {
        const T c1 = (T)0.30901699437494742410;
        const T c2 = (T)-0.80901699437494742410;
        const T s1 = (T)0.95105651629515357212;
        const T s2 = (T)0.58778525229247312917;
        cx<T> t1 = cadd(v[1], v[4]), d1 = csub(v[1], v[4]);
        cx<T> t2 = cadd(v[2], v[3]), d2 = csub(v[2], v[3]);
        cx<T> a1 = mk<T>(v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y);
        cx<T> a2 = mk<T>(v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y);
        cx<T> e1 = mk<T>(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y);
        cx<T> e2 = mk<T>(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y);
        cx<T> b1 = mk<T>(-s * e1.y, s * e1.x);
        cx<T> b2 = mk<T>(-s * e2.y, s * e2.x);
        v[0] = cadd(v[0], cadd(t1, t2));
        v[1] = cadd(a1, b1);
        v[4] = csub(a1, b1);
        v[2] = cadd(a2, b2);
        v[3] = csub(a2, b2);
    }
}

// One Stockham stage in registers: in -> out, span NS so far, radix R; twiddles
// exp(SIGN 2 pi i m / N) from the compile-time table.
template <typename T, int N, int NS, int R, int SIGN>
__device__ __forceinline__ void line_stage(const cx<T>* in, cx<T>* out) {
    constexpr int NBF = N / R;
    constexpr int TS = N / (NS * R);
#pragma unroll
    for (int j = 0; j < NBF; ++j) {
        const int k = j % NS;
        cx<T> v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = in[j + r * NBF];
        if (k != 0) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const int m = r * k * TS;
                const cx<T> w = mk<T>((T)kRoots<N>.c[m], (T)(SIGN < 0 ? -kRoots<N>.s[m] : kRoots<N>.s[m]));
                v[r] = cmul(v[r], w);
            }
        }
        bfly<T, R, SIGN>(v);
        const int o = (j / NS) * NS * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) out[o + r * NS] = v[r];
    }
}

template <typename T, int N, int S, int NS, int SIGN>
__device__ __forceinline__ void line_fft_rec(cx<T>* a, cx<T>* b) {
    constexpr RadixPlan P = LinePlan<N>::p;
    if constexpr (S < P.nr) {
        constexpr int R = P.rad[S];
        line_stage<T, N, NS, R, SIGN>(a, b);
        line_fft_rec<T, N, S + 1, NS * R, SIGN>(b, a);
    }
}

// in-place transform of v[N] (result back in v)
template <typename T, int N, int SIGN>
__device__ __forceinline__ void line_fft(cx<T>* v) {
    cx<T> tmp[N];
    line_fft_rec<T, N, 0, 1, SIGN>(v, tmp);
    constexpr RadixPlan P = LinePlan<N>::p;
    if constexpr (P.nr % 2 == 1) {
#pragma unroll
        for (int e = 0; e < N; ++e) v[e] = tmp[e];
    }
}

}  // namespace fftl
}  // namespace mb
