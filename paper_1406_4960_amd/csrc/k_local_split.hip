// Local-potential part of H c for in-plane grids too large for one FFT line per
// thread (same operation as k_local.hip):
//   evaluate psi(G, z_q) = sum_t B_{s-1+t}(z_q) c(G, s-1+t) on each Gauss plane of
//   interval s, scatter, inverse 2D FFT, multiply by V(rho, z_q), forward 2D FFT,
//   gather, project onto the kappa spline rows of interval s (local-potential matrix
//   elements of Sec. II.B.1, taken on the grid).
// Each line of length N = A B is transformed in two register steps through LDS:
//   inverse (decimation in frequency): A-point transforms over a for each b of
//     x[b + B a], twiddle exp(+2 pi i b k_a / N), then B-point transforms over b of the
//     contiguous groups; the result X[k_a + A k_b] is left at position B k_a + k_b;
//   forward (decimation in time) reads that order back: B-point transforms of the
//     contiguous groups, twiddle exp(-2 pi i a k_1 / N), A-point transforms with stride B,
//     natural order out.
// So the permutation left by the inverse transform is undone by the forward one; the
// potential multiply in between reads V at the permuted (logical) index.  One
// workgroup owns one band and one knot interval and runs its planes one after another
// (row stride N2 + 1 in LDS).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "cplx.h"
#include "fft_line.h"
#include "mbks_internal.h"

namespace mb {

namespace {

constexpr int KORD = 4;
using fftl::kRoots;
using fftl::line_fft;

// N = A B with B the largest divisor not above sqrt(N)
constexpr int split_b(int n) {
    int b = 1;
    for (int d = 1; d * d <= n; ++d)
        if (n % d == 0) b = d;
    return b;
}

template <int N>
struct Split {
    static constexpr int B = split_b(N);
    static constexpr int A = N / B;
};

template <typename T, int N>
__device__ __forceinline__ cx<T> root(int e, int sign) {
    const double c = kRoots<N>.c[e], s = kRoots<N>.s[e];
    return mk<T>((T)c, (T)(sign < 0 ? -s : s));
}

// position of logical index k along an axis after the inverse transform
template <int N>
__device__ __forceinline__ int logical_of(int p) {
    constexpr int A = Split<N>::A, B = Split<N>::B;
    return p / B + A * (p % B);
}

// inverse transform, step 1: task (line, b)
template <typename T, int N>
__device__ __forceinline__ void inv_step1(cx<T>* base, int st, int b) {
    constexpr int A = Split<N>::A, B = Split<N>::B;
    cx<T> v[A];
#pragma unroll
    for (int a = 0; a < A; ++a) v[a] = base[(b + B * a) * st];
    line_fft<T, A, +1>(v);
#pragma unroll
    for (int k = 1; k < A; ++k) v[k] = cmul(v[k], root<T, N>((b * k) % N, +1));
#pragma unroll
    for (int k = 0; k < A; ++k) base[(b + B * k) * st] = v[k];
}

// inverse transform, step 2: task (line, k_a)
template <typename T, int N>
__device__ __forceinline__ void inv_step2(cx<T>* base, int st, int ka) {
    constexpr int B = Split<N>::B;
    cx<T> u[B];
#pragma unroll
    for (int b = 0; b < B; ++b) u[b] = base[(B * ka + b) * st];
    line_fft<T, B, +1>(u);
#pragma unroll
    for (int k = 0; k < B; ++k) base[(B * ka + k) * st] = u[k];
}

// forward transform, step 1: task (line, a); optional real factors w[b] applied first
template <typename T, int N>
__device__ __forceinline__ void fwd_step1(cx<T>* base, int st, int a, const T* w) {
    constexpr int B = Split<N>::B;
    cx<T> u[B];
#pragma unroll
    for (int b = 0; b < B; ++b) u[b] = base[(B * a + b) * st];
    if (w) {
#pragma unroll
        for (int b = 0; b < B; ++b) u[b] = mk<T>(u[b].x * w[b], u[b].y * w[b]);
    }
    line_fft<T, B, -1>(u);
#pragma unroll
    for (int k = 1; k < B; ++k) u[k] = cmul(u[k], root<T, N>((a * k) % N, -1));
#pragma unroll
    for (int k = 0; k < B; ++k) base[(B * a + k) * st] = u[k];
}

// forward transform, step 2: task (line, k_1)
template <typename T, int N>
__device__ __forceinline__ void fwd_step2(cx<T>* base, int st, int k1) {
    constexpr int A = Split<N>::A, B = Split<N>::B;
    cx<T> v[A];
#pragma unroll
    for (int a = 0; a < A; ++a) v[a] = base[(B * a + k1) * st];
    line_fft<T, A, -1>(v);
#pragma unroll
    for (int k = 0; k < A; ++k) base[(B * k + k1) * st] = v[k];
}

template <typename TI, typename T>
struct SplitArgs {
    const cx<TI>* c;
    cx<T>* part;
    const T* bval;
    const T* wbval;
    const T* V;
    const int32_t* gmap;
    const int32_t* rows;
    int nbands, ld, ng, nint, nq, nb, nrows;
    T inv_n;
};

template <int N1>
constexpr size_t SPLIT_HDR = ((sizeof(int32_t) * N1 + 255) / 256) * 256;

template <typename T, int N1, int N2>
constexpr size_t split_lds() {
    return SPLIT_HDR<N1> + sizeof(cx<T>) * (size_t)N1 * (N2 + 1);
}

// items == nullptr: one problem described by a0; otherwise a batch of problems with the
// same grid, item t owning work units [unit_begin[t], unit_begin[t+1]).
template <typename TI, typename T, int N1, int N2, int NT, int MAXG>
__global__ __launch_bounds__(NT) void k_local_split(SplitArgs<TI, T> a0, const SplitArgs<TI, T>* items,
                                                    const int32_t* unit_begin, int nitems) {
    constexpr int P2 = N2 + 1;
    constexpr int A1 = Split<N1>::A, B1 = Split<N1>::B;
    constexpr int A2 = Split<N2>::A, B2 = Split<N2>::B;
    extern __shared__ unsigned char smem_raw[];
    int32_t* rows = reinterpret_cast<int32_t*>(smem_raw);
    cx<T>* grid = reinterpret_cast<cx<T>*>(smem_raw + SPLIT_HDR<N1>);

    unsigned L = xcd_logical(blockIdx.x, gridDim.x);
    SplitArgs<TI, T> a = a0;
    if (items) {
        const int it = batch_item_of(unit_begin, nitems, L);
        a = items[it];
        L -= (unsigned)unit_begin[it];
    }
    const int b = (int)(L % (unsigned)a.nbands);
    const int s = (int)(L / (unsigned)a.nbands);
    if (s >= a.nint) return;
    const int tid = threadIdx.x;
    for (int e = tid; e < a.nrows; e += NT) rows[e] = a.rows[e];

    const cx<TI>* cb = a.c + (size_t)b * a.nb * a.ld;
    cx<T> acc[KORD][MAXG];
    int off[MAXG];
#pragma unroll
    for (int k = 0; k < MAXG; ++k) {
        const int g = tid + k * NT;
        off[k] = 0;
        if (g < a.ng) {
            const int gm = a.gmap[g];
            off[k] = (gm / N2) * P2 + (gm % N2);
        }
#pragma unroll
        for (int t = 0; t < KORD; ++t) acc[t][k] = mk<T>(0, 0);
    }
    const int nr = a.nrows;

    for (int jq = 0; jq < a.nq; ++jq) {
        const int q = s * a.nq + jq;
        for (int e = tid; e < N1 * P2; e += NT) grid[e] = mk<T>(0, 0);
        __syncthreads();
        // evaluate and scatter
        {
            T bv[KORD];
#pragma unroll
            for (int t = 0; t < KORD; ++t) bv[t] = a.bval[(size_t)q * KORD + t];
#pragma unroll
            for (int k = 0; k < MAXG; ++k) {
                const int g = tid + k * NT;
                if (g < a.ng) {
                    cx<T> psi = mk<T>(0, 0);
#pragma unroll
                    for (int t = 0; t < KORD; ++t) {
                        const int row = s - 1 + t;
                        if (row >= 0 && row < a.nb) {
                            const cx<TI> v = cb[(size_t)row * a.ld + g];
                            psi.x = fma(bv[t], (T)v.x, psi.x);
                            psi.y = fma(bv[t], (T)v.y, psi.y);
                        }
                    }
                    grid[off[k]] = psi;
                }
            }
        }
        __syncthreads();
        // inverse transform along the rows that hold G (lines = rows[], stride 1)
        for (int t = tid; t < nr * B2; t += NT) {
            const int r = t % nr, sub = t / nr;
            inv_step1<T, N2>(grid + rows[r] * P2, 1, sub);
        }
        __syncthreads();
        for (int t = tid; t < nr * A2; t += NT) {
            const int r = t % nr, sub = t / nr;
            inv_step2<T, N2>(grid + rows[r] * P2, 1, sub);
        }
        __syncthreads();
        // inverse transform along every column (stride P2)
        for (int t = tid; t < N2 * B1; t += NT) {
            const int col = t % N2, sub = t / N2;
            inv_step1<T, N1>(grid + col, P2, sub);
        }
        __syncthreads();
        for (int t = tid; t < N2 * A1; t += NT) {
            const int col = t % N2, sub = t / N2;
            inv_step2<T, N1>(grid + col, P2, sub);
        }
        __syncthreads();
        // potential multiply fused into the first forward column step: element at
        // position (B1 a + k, col) holds logical row logical_of<N1>(B1 a + k) and
        // logical column logical_of<N2>(col)
        const T* Vq = a.V + (size_t)q * (N1 * N2);
        for (int t = tid; t < N2 * A1; t += NT) {
            const int col = t % N2, sub = t / N2;
            const int j2 = logical_of<N2>(col);
            T w[B1];
#pragma unroll
            for (int k = 0; k < B1; ++k) w[k] = Vq[logical_of<N1>(B1 * sub + k) * N2 + j2];
            fwd_step1<T, N1>(grid + col, P2, sub, w);
        }
        __syncthreads();
        for (int t = tid; t < N2 * B1; t += NT) {
            const int col = t % N2, sub = t / N2;
            fwd_step2<T, N1>(grid + col, P2, sub);
        }
        __syncthreads();
        // forward transform along the rows that hold G
        for (int t = tid; t < nr * A2; t += NT) {
            const int r = t % nr, sub = t / nr;
            fwd_step1<T, N2>(grid + rows[r] * P2, 1, sub, (const T*)nullptr);
        }
        __syncthreads();
        for (int t = tid; t < nr * B2; t += NT) {
            const int r = t % nr, sub = t / nr;
            fwd_step2<T, N2>(grid + rows[r] * P2, 1, sub);
        }
        __syncthreads();
        // gather and project
        T wb[KORD];
#pragma unroll
        for (int t = 0; t < KORD; ++t) wb[t] = a.wbval[(size_t)q * KORD + t] * a.inv_n;
#pragma unroll
        for (int k = 0; k < MAXG; ++k) {
            const int g = tid + k * NT;
            if (g < a.ng) {
                const cx<T> u = grid[off[k]];
#pragma unroll
                for (int t = 0; t < KORD; ++t) {
                    acc[t][k].x = fma(wb[t], u.x, acc[t][k].x);
                    acc[t][k].y = fma(wb[t], u.y, acc[t][k].y);
                }
            }
        }
        __syncthreads();
    }
    cx<T>* pb = a.part + ((size_t)b * a.nint + s) * KORD * a.ld;
#pragma unroll
    for (int k = 0; k < MAXG; ++k) {
        const int g = tid + k * NT;
        if (g < a.ng) {
#pragma unroll
            for (int t = 0; t < KORD; ++t) pb[(size_t)t * a.ld + g] = acc[t][k];
        }
    }
}

template <typename TI, typename T, int N1, int N2>
SplitArgs<TI, T> make_split_args(Problem* p, int ik, const void* c, void* part, int nbands, int ld) {
    const KPoint& kp = p->kp[ik];
    const bool dbl = sizeof(T) == 8;
    SplitArgs<TI, T> a;
    a.c = (const cx<TI>*)c;
    a.part = (cx<T>*)part;
    a.bval = (const T*)(dbl ? (const void*)p->d_bval : (const void*)p->d_bvalf);
    a.wbval = (const T*)(dbl ? (const void*)p->d_wbval : (const void*)p->d_wbvalf);
    a.V = (const T*)(dbl ? (const void*)p->d_V : (const void*)p->d_Vf);
    a.gmap = kp.d_gmap;
    a.rows = kp.d_rows;
    a.nbands = nbands;
    a.ld = ld;
    a.ng = kp.ng;
    a.nint = p->nint;
    a.nq = p->nq;
    a.nb = p->nb;
    a.nrows = (int)kp.rows.size();
    a.inv_n = (T)(1.0 / ((double)N1 * N2));
    return a;
}

// threads per workgroup: FP64 planes take most of the LDS (one workgroup per CU), so
// more threads; FP32 planes leave room for two or three workgroups per CU
template <typename T>
constexpr int split_threads() { return sizeof(T) == 8 ? 512 : 256; }

template <int N1, int N2, int NT>
constexpr int split_maxg() { return (N1 * N2 * 11 / 20 + NT - 1) / NT; }

template <typename TI, typename T, int N1, int N2>
mb_status split_launch(const std::vector<SplitArgs<TI, T>>& args, const std::vector<int32_t>& begin, int units,
                       int64_t bands, TableUploader* up, hipStream_t s) {
    constexpr int NT = split_threads<T>();
    constexpr int MAXG = split_maxg<N1, N2, NT>();
    constexpr size_t lds = split_lds<T, N1, N2>();
    static_assert(lds <= 163840, "grid does not fit in LDS");
    auto kern = k_local_split<TI, T, N1, N2, NT, MAXG>;
    if (lds > 65536)
        MB_HIP_TRY(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const SplitArgs<TI, T>* dargs = nullptr;
    const int32_t* dbegin = nullptr;
    if (up) {
        void *ha, *da, *hb, *db;
        if (!up->reserve(args.size() * sizeof(args[0]), &ha, &da) || !up->reserve(begin.size() * 4, &hb, &db))
            return set_error(MB_ERR_OOM, "batch descriptor table full");
        std::memcpy(ha, args.data(), args.size() * sizeof(args[0]));
        std::memcpy(hb, begin.data(), begin.size() * 4);
        MB_HIP_TRY(hipMemcpyAsync(da, ha, args.size() * sizeof(args[0]), hipMemcpyHostToDevice, s));
        MB_HIP_TRY(hipMemcpyAsync(db, hb, begin.size() * 4, hipMemcpyHostToDevice, s));
        dargs = (const SplitArgs<TI, T>*)da;
        dbegin = (const int32_t*)db;
    }
    StageScope ts_(sizeof(T) == 8 ? MB_STAGE_LOCAL : MB_STAGE_LOCAL32, s, bands);
    hipLaunchKernelGGL(kern, dim3((unsigned)units), dim3(NT), lds, s, args[0], dargs, dbegin,
                       up ? (int)args.size() : 0);
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

template <typename TI, typename T, int N1, int N2>
mb_status split_impl(const std::vector<BatchItem>& items, TableUploader* up, hipStream_t s) {
    constexpr int NT = split_threads<T>();
    constexpr int MAXG = split_maxg<N1, N2, NT>();
    std::vector<SplitArgs<TI, T>> args;
    std::vector<int32_t> begin;
    int units = 0;
    int64_t bands = 0;
    for (const auto& it : items) {
        if (it.p->order != KORD || it.p->N1 != N1 || it.p->N2 != N2) return MB_ERR_INVALID_ARG;
        if (it.p->kp[it.ik].ng > NT * MAXG) return MB_ERR_INVALID_ARG;
        if (it.nbands == 0) continue;
        args.push_back(make_split_args<TI, T, N1, N2>(it.p, it.ik, it.c, it.part, it.nbands, it.ld));
        begin.push_back(units);
        units += it.nbands * it.p->nint;
        bands += it.nbands;
    }
    if (units == 0) return MB_OK;
    return split_launch<TI, T, N1, N2>(args, begin, units, bands, up, s);
}

template <typename TI, typename T>
mb_status split_by_size(const std::vector<BatchItem>& items, TableUploader* up, hipStream_t s) {
    const Problem* p0 = items[0].p;
    const int n1 = p0->N1, n2 = p0->N2;
    if (n1 == 128 && n2 == 64) {
        // FP32 planes of this grid run on the generic kernel: the two-step kernel's
        // FP32 instantiation for it failed its comparison with the generic kernel and
        // is switched off until the cause is found
        if constexpr (sizeof(T) == 8) return split_impl<TI, T, 128, 64>(items, up, s);
        return MB_ERR_INVALID_ARG;
    }
    if (n1 != n2) return MB_ERR_INVALID_ARG;
    switch (n1) {
        case 72: return split_impl<TI, T, 72, 72>(items, up, s);
        case 75: return split_impl<TI, T, 75, 75>(items, up, s);
        case 80: return split_impl<TI, T, 80, 80>(items, up, s);
        default: break;
    }
    if constexpr (sizeof(T) == 8) {
        // FP32 grids up to 64 go to the line kernel
        switch (n1) {
            case 45: return split_impl<TI, T, 45, 45>(items, up, s);
            case 48: return split_impl<TI, T, 48, 48>(items, up, s);
            case 50: return split_impl<TI, T, 50, 50>(items, up, s);
            case 54: return split_impl<TI, T, 54, 54>(items, up, s);
            case 60: return split_impl<TI, T, 60, 60>(items, up, s);
            case 64: return split_impl<TI, T, 64, 64>(items, up, s);
            default: break;
        }
    }
    return MB_ERR_INVALID_ARG;
}

mb_status split_dispatch(const std::vector<BatchItem>& items, int prec, TableUploader* up, hipStream_t s) {
    if (items.empty()) return MB_OK;
    if (prec == 0) return split_by_size<double, double>(items, up, s);
    if (prec == 1) return split_by_size<float, float>(items, up, s);
    return split_by_size<double, float>(items, up, s);
}

}  // namespace

// Returns MB_ERR_INVALID_ARG (no message) if the grid has no split kernel.
mb_status launch_local_split(Problem* p, int ik, const void* c, void* part, int nbands, int ld, int prec,
                             hipStream_t s) {
    std::vector<BatchItem> one{BatchItem{p, ik, c, nullptr, part, nullptr, nbands, ld}};
    return split_dispatch(one, prec, nullptr, s);
}

// items must share the in-plane grid
mb_status launch_local_split_batch(const std::vector<BatchItem>& items, int prec, TableUploader& up,
                                   hipStream_t s) {
    return split_dispatch(items, prec, &up, s);
}

}  // namespace mb
