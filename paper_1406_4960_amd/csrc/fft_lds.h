// In-place mixed-radix (2, 3, 4, 5) Stockham transforms of grid lines held in LDS, shared
// by the kernels that take whole in-plane grid planes through LDS.
#pragma once

#include <algorithm>

#include "cplx.h"
#include "mbks_internal.h"

namespace mb {

constexpr int MAXB = 4;  // butterflies per thread per FFT stage

// y_k = sum_r v_r exp(sign 2 pi i r k / R) for R in {2, 3, 4, 5}
template <typename T, int R>
__device__ inline void butterfly(cx<T>* v, int sign) {
    if constexpr (R == 2) {
        cx<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 4) {
        cx<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        cx<T> t2 = cadd(v[1], v[3]), d = csub(v[1], v[3]);
        T s = (T)sign;
        cx<T> t3 = mk<T>(-s * d.y, s * d.x);  // (sign i) * d
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    } else if constexpr (R == 3) {
        const T c3 = (T)-0.5;
        const T s3 = (T)0.86602540378443864676;  // sqrt(3)/2
        cx<T> t = cadd(v[1], v[2]), d = csub(v[1], v[2]);
        cx<T> a = mk<T>(v[0].x + c3 * t.x, v[0].y + c3 * t.y);
        T ss = (T)sign * s3;
        cx<T> b = mk<T>(-ss * d.y, ss * d.x);
        v[0] = cadd(v[0], t);
        v[1] = cadd(a, b);
        v[2] = csub(a, b);
    } else if constexpr (R == 5) {
        const T c1 = (T)0.30901699437494742410;   // cos(2 pi / 5) = (sqrt 5 - 1) / 4
        const T c2 = (T)-0.80901699437494742410;  // cos(4 pi / 5) = -(sqrt 5 + 1) / 4
        const T s1 = (T)0.95105651629515357212;   // sin(2 pi / 5)
        const T s2 = (T)0.58778525229247312917;   // sin(4 pi / 5)
        cx<T> t1 = cadd(v[1], v[4]), d1 = csub(v[1], v[4]);
        cx<T> t2 = cadd(v[2], v[3]), d2 = csub(v[2], v[3]);
        T s = (T)sign;
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

// One Stockham radix-R stage over `nlines` lines of length n held in LDS, in
// place: every thread first loads its butterflies' inputs, the block
// synchronises, then twiddles, transforms and stores.
template <typename T, int NT, int R>
__device__ inline void fft_stage(cx<T>* buf, const cx<T>* tw, int n, int Ns, int nlines,
                                 const int32_t* rows, int rowmul, int stride, int sign) {
    const int nbf = n / R;
    const int total = nlines * nbf;
    const int twstep = n / (Ns * R);
    cx<T> v[MAXB][R];
    int base[MAXB], jj[MAXB];
#pragma unroll
    for (int kk = 0; kk < MAXB; ++kk) {
        int idx = threadIdx.x + kk * NT;
        if (idx < total) {
            int line = idx / nbf;
            int j = idx - line * nbf;
            int b = (rows ? rows[line] : line) * rowmul;
            base[kk] = b;
            jj[kk] = j;
#pragma unroll
            for (int r = 0; r < R; ++r) v[kk][r] = buf[b + (j + r * nbf) * stride];
        }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < MAXB; ++kk) {
        int idx = threadIdx.x + kk * NT;
        if (idx < total) {
            int j = jj[kk];
            int k = j % Ns;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                cx<T> w = tw[r * k * twstep];
                if (sign < 0) w.y = -w.y;
                v[kk][r] = cmul(v[kk][r], w);
            }
            butterfly<T, R>(v[kk], sign);
            int o = (j / Ns) * Ns * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[base[kk] + (o + r * Ns) * stride] = v[kk][r];
        }
    }
    __syncthreads();
}

template <typename T, int NT>
__device__ void fft_axis(cx<T>* buf, const cx<T>* tw, const FftPlan& pl, int nlines,
                         const int32_t* rows, int rowmul, int stride, int sign) {
    int Ns = 1;
    for (int st = 0; st < pl.nr; ++st) {
        int R = pl.rad[st];
        switch (R) {
            case 2: fft_stage<T, NT, 2>(buf, tw, pl.n, Ns, nlines, rows, rowmul, stride, sign); break;
            case 3: fft_stage<T, NT, 3>(buf, tw, pl.n, Ns, nlines, rows, rowmul, stride, sign); break;
            case 4: fft_stage<T, NT, 4>(buf, tw, pl.n, Ns, nlines, rows, rowmul, stride, sign); break;
            default: fft_stage<T, NT, 5>(buf, tw, pl.n, Ns, nlines, rows, rowmul, stride, sign); break;
        }
        Ns *= R;
    }
}

// largest number of butterflies of one stage over nlines lines of the plan's length
inline int max_stage_work(const FftPlan& pl, int nlines) {
    int w = 0;
    for (int st = 0; st < pl.nr; ++st) w = std::max(w, nlines * (pl.n / pl.rad[st]));
    return w;
}

}  // namespace mb
