// Local-potential part of H c for in-plane grids small enough that one thread
// can hold a whole FFT line in registers (same operation as k_local.hip):
//   evaluate psi(G, z_q) = sum_t B_{s-1+t}(z_q) c(G, s-1+t) for a group of Gauss
//   planes of interval s, scatter, inverse 2D FFT, multiply by V(rho, z_q),
//   forward 2D FFT, gather, project onto the kappa spline rows of interval s
//   (local-potential matrix elements of Sec. II.B.1, taken on the grid).
// Each workgroup owns one band and one knot interval and keeps a group of planes
// in LDS (row stride N2 + 1).  Transforms run line by line: a thread loads a row
// or a column, runs a compile-time mixed-radix Stockham FFT in registers and
// stores it back, so a plane costs four passes through LDS instead of one per
// radix stage.  The column pass fuses inverse FFT, V multiply and forward FFT.
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
using fftl::line_fft;

// LDS bytes ahead of the planes: the list of grid rows that hold sphere points
template <int N1>
constexpr size_t LINE_HDR = ((sizeof(int32_t) * N1 + 255) / 256) * 256;

template <typename TI, typename T>
struct LineArgs {
    const cx<TI>* c;
    cx<T>* part;
    const T* bval;
    const T* wbval;
    const T* V;
    const int32_t* gmap;
    const int32_t* rows;
    int nbands, ld, ng, nint, nq, nb, nrows, qp;
    T inv_n;
};

// item of a batched launch holding flat work unit u (unit_begin ascending, n items)
// items == nullptr: one problem described by a0; otherwise a batch of problems with the
// same grid, item t owning work units [unit_begin[t], unit_begin[t+1]).
template <typename TI, typename T, int N1, int N2, int NT, int MAXG>
__global__ __launch_bounds__(NT) void k_local_lines(LineArgs<TI, T> a0, const LineArgs<TI, T>* items,
                                                    const int32_t* unit_begin, int nitems) {
    constexpr int P2 = N2 + 1;          // padded row stride
    constexpr int PLANE = N1 * P2;
    extern __shared__ unsigned char smem_raw[];
    int32_t* rows = reinterpret_cast<int32_t*>(smem_raw);
    cx<T>* grid = reinterpret_cast<cx<T>*>(smem_raw + LINE_HDR<N1>);

    unsigned L = xcd_logical(blockIdx.x, gridDim.x);
    LineArgs<TI, T> a = a0;
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
#pragma unroll
    for (int t = 0; t < KORD; ++t)
#pragma unroll
        for (int k = 0; k < MAXG; ++k) acc[t][k] = mk<T>(0, 0);

    for (int q0 = 0; q0 < a.nq; q0 += a.qp) {
        const int np = min(a.qp, a.nq - q0);
        // zero the planes of this group
        for (int e = tid; e < np * PLANE; e += NT) grid[e] = mk<T>(0, 0);
        __syncthreads();
        // evaluate and scatter: c rows s-1 .. s+2 read once for all planes of the group
#pragma unroll
        for (int k = 0; k < MAXG; ++k) {
            const int g = tid + k * NT;
            if (g < a.ng) {
                cx<T> cv[KORD];
#pragma unroll
                for (int t = 0; t < KORD; ++t) {
                    const int row = s - 1 + t;
                    if (row >= 0 && row < a.nb) {
                        cx<TI> v = cb[(size_t)row * a.ld + g];
                        cv[t] = mk<T>((T)v.x, (T)v.y);
                    } else {
                        cv[t] = mk<T>(0, 0);
                    }
                }
                const int gm = a.gmap[g];
                const int off = (gm / N2) * P2 + (gm % N2);
                for (int jq = 0; jq < np; ++jq) {
                    const T* bv = a.bval + (size_t)(s * a.nq + q0 + jq) * KORD;
                    cx<T> psi = mk<T>(0, 0);
#pragma unroll
                    for (int t = 0; t < KORD; ++t) {
                        psi.x = fma(bv[t], cv[t].x, psi.x);
                        psi.y = fma(bv[t], cv[t].y, psi.y);
                    }
                    grid[jq * PLANE + off] = psi;
                }
            }
        }
        __syncthreads();
        // inverse transform along rows that hold G
        for (int line = tid; line < np * a.nrows; line += NT) {
            const int jq = line / a.nrows;
            cx<T>* base = grid + jq * PLANE + rows[line - jq * a.nrows] * P2;
            cx<T> v[N2];
#pragma unroll
            for (int e = 0; e < N2; ++e) v[e] = base[e];
            line_fft<T, N2, +1>(v);
#pragma unroll
            for (int e = 0; e < N2; ++e) base[e] = v[e];
        }
        __syncthreads();
        // columns: inverse FFT, multiply by V(rho, z_q), forward FFT
        for (int line = tid; line < np * N2; line += NT) {
            const int jq = line / N2;
            const int j2 = line - jq * N2;
            cx<T>* base = grid + jq * PLANE + j2;
            const T* Vq = a.V + (size_t)(s * a.nq + q0 + jq) * (N1 * N2) + j2;
            cx<T> v[N1];
#pragma unroll
            for (int e = 0; e < N1; ++e) v[e] = base[e * P2];
            line_fft<T, N1, +1>(v);
#pragma unroll
            for (int e = 0; e < N1; ++e) {
                const T w = Vq[e * N2];
                v[e] = mk<T>(v[e].x * w, v[e].y * w);
            }
            line_fft<T, N1, -1>(v);
#pragma unroll
            for (int e = 0; e < N1; ++e) base[e * P2] = v[e];
        }
        __syncthreads();
        // forward transform along rows that hold G
        for (int line = tid; line < np * a.nrows; line += NT) {
            const int jq = line / a.nrows;
            cx<T>* base = grid + jq * PLANE + rows[line - jq * a.nrows] * P2;
            cx<T> v[N2];
#pragma unroll
            for (int e = 0; e < N2; ++e) v[e] = base[e];
            line_fft<T, N2, -1>(v);
#pragma unroll
            for (int e = 0; e < N2; ++e) base[e] = v[e];
        }
        __syncthreads();
        // gather and project onto the kappa rows of the interval
#pragma unroll
        for (int k = 0; k < MAXG; ++k) {
            const int g = tid + k * NT;
            if (g < a.ng) {
                const int gm = a.gmap[g];
                const int off = (gm / N2) * P2 + (gm % N2);
                for (int jq = 0; jq < np; ++jq) {
                    const cx<T> u = grid[jq * PLANE + off];
                    const T* wb = a.wbval + (size_t)(s * a.nq + q0 + jq) * KORD;
#pragma unroll
                    for (int t = 0; t < KORD; ++t) {
                        const T w = wb[t] * a.inv_n;
                        acc[t][k].x = fma(w, u.x, acc[t][k].x);
                        acc[t][k].y = fma(w, u.y, acc[t][k].y);
                    }
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
LineArgs<TI, T> make_line_args(Problem* p, int ik, const void* c, void* part, int nbands, int ld, int qp) {
    const KPoint& kp = p->kp[ik];
    const bool dbl = sizeof(T) == 8;
    LineArgs<TI, T> a;
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
    a.qp = qp;
    a.inv_n = (T)(1.0 / ((double)N1 * N2));
    return a;
}

// planes per group: all Gauss planes of an interval when they fit in the LDS budget
template <typename T, int N1, int N2>
int planes_per_group(int nq, size_t budget, size_t* lds_out) {
    const size_t hdr = LINE_HDR<N1>;
    const size_t plane = sizeof(cx<T>) * (size_t)N1 * (N2 + 1);
    int qp = nq;
    while (qp > 1 && hdr + qp * plane > budget) --qp;
    *lds_out = hdr + qp * plane;
    return qp;
}

template <typename TI, typename T, int N1, int N2, int NT, int MAXG>
mb_status run_lines(Problem* p, int ik, const void* c, void* part, int nbands, int ld, hipStream_t s, int qp,
                    size_t lds) {
    const KPoint& kp = p->kp[ik];
    const bool dbl = sizeof(T) == 8;
    LineArgs<TI, T> a;
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
    a.qp = qp;
    a.inv_n = (T)(1.0 / ((double)N1 * N2));
    auto kern = k_local_lines<TI, T, N1, N2, NT, MAXG>;
    if (lds > 65536)
        MB_HIP_TRY(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    unsigned nblocks = (unsigned)nbands * (unsigned)p->nint;
    StageScope ts_(sizeof(T) == 8 ? MB_STAGE_LOCAL : MB_STAGE_LOCAL32, s, nbands);
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(NT), lds, s, a, (const LineArgs<TI, T>*)nullptr,
                       (const int32_t*)nullptr, 0);
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

// planes per group: all Gauss planes of an interval when they fit in `budget` bytes of LDS
template <typename TI, typename T, int N1, int N2>
mb_status lines_dispatch(Problem* p, int ik, const void* c, void* part, int nbands, int ld, hipStream_t s,
                         size_t budget) {
    const size_t hdr = LINE_HDR<N1>;
    const size_t plane = sizeof(cx<T>) * (size_t)N1 * (N2 + 1);
    int qp = p->nq;
    while (qp > 1 && hdr + qp * plane > budget) --qp;
    const size_t lds = hdr + qp * plane;
    if (lds > 163840) return MB_ERR_INVALID_ARG;
    // accumulator slots for G sets up to 0.55 of the grid; larger sets use the generic kernel
    constexpr int MAXG = (N1 * N2 * 11 / 20 + 255) / 256;
    if (p->kp[ik].ng > 256 * MAXG) return MB_ERR_INVALID_ARG;
    return run_lines<TI, T, N1, N2, 256, MAXG>(p, ik, c, part, nbands, ld, s, qp, lds);
}

template <typename TI, typename T>
mb_status lines_by_size(Problem* p, int ik, const void* c, void* part, int nbands, int ld, hipStream_t s,
                        int budget_kb) {
    if (p->N1 != p->N2) return MB_ERR_INVALID_ARG;
    const size_t budget = (size_t)budget_kb * 1024;
    switch (p->N1) {
        case 16: return lines_dispatch<TI, T, 16, 16>(p, ik, c, part, nbands, ld, s, budget);
        case 24: return lines_dispatch<TI, T, 24, 24>(p, ik, c, part, nbands, ld, s, budget);
        case 25: return lines_dispatch<TI, T, 25, 25>(p, ik, c, part, nbands, ld, s, budget);
        case 27: return lines_dispatch<TI, T, 27, 27>(p, ik, c, part, nbands, ld, s, budget);
        case 30: return lines_dispatch<TI, T, 30, 30>(p, ik, c, part, nbands, ld, s, budget);
        case 32: return lines_dispatch<TI, T, 32, 32>(p, ik, c, part, nbands, ld, s, budget);
        case 36: return lines_dispatch<TI, T, 36, 36>(p, ik, c, part, nbands, ld, s, budget);
        case 40: return lines_dispatch<TI, T, 40, 40>(p, ik, c, part, nbands, ld, s, budget);
        default: break;
    }
    if constexpr (sizeof(T) == 4) {
        switch (p->N1) {
            case 45: return lines_dispatch<TI, T, 45, 45>(p, ik, c, part, nbands, ld, s, budget);
            case 48: return lines_dispatch<TI, T, 48, 48>(p, ik, c, part, nbands, ld, s, budget);
            case 50: return lines_dispatch<TI, T, 50, 50>(p, ik, c, part, nbands, ld, s, budget);
            case 54: return lines_dispatch<TI, T, 54, 54>(p, ik, c, part, nbands, ld, s, budget);
            case 60: return lines_dispatch<TI, T, 60, 60>(p, ik, c, part, nbands, ld, s, budget);
            case 64: return lines_dispatch<TI, T, 64, 64>(p, ik, c, part, nbands, ld, s, budget);
            default: break;
        }
    }
    return MB_ERR_INVALID_ARG;
}

template <typename TI, typename T, int N1, int N2>
mb_status lines_batch_impl(const std::vector<BatchItem>& items, TableUploader& up, hipStream_t s) {
    constexpr int MAXG = (N1 * N2 * 11 / 20 + 255) / 256;
    const size_t budget = 110 * 1024;
    std::vector<LineArgs<TI, T>> args;
    std::vector<int32_t> begin;
    size_t lds = 0;
    int units = 0;
    for (const auto& it : items) {
        if (it.p->kp[it.ik].ng > 256 * MAXG || it.p->order != KORD) return MB_ERR_INVALID_ARG;
        size_t l = 0;
        const int qp = planes_per_group<T, N1, N2>(it.p->nq, budget, &l);
        lds = std::max(lds, l);
        args.push_back(make_line_args<TI, T, N1, N2>(it.p, it.ik, it.c, it.part, it.nbands, it.ld, qp));
        begin.push_back(units);
        units += it.nbands * it.p->nint;
    }
    if (units == 0) return MB_OK;
    void *ha, *da, *hb, *db;
    if (!up.reserve(args.size() * sizeof(args[0]), &ha, &da) || !up.reserve(begin.size() * 4, &hb, &db))
        return set_error(MB_ERR_OOM, "batch descriptor table full");
    std::memcpy(ha, args.data(), args.size() * sizeof(args[0]));
    std::memcpy(hb, begin.data(), begin.size() * 4);
    MB_HIP_TRY(hipMemcpyAsync(da, ha, args.size() * sizeof(args[0]), hipMemcpyHostToDevice, s));
    MB_HIP_TRY(hipMemcpyAsync(db, hb, begin.size() * 4, hipMemcpyHostToDevice, s));
    auto kern = k_local_lines<TI, T, N1, N2, 256, MAXG>;
    if (lds > 65536)
        MB_HIP_TRY(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int64_t tot_bands = 0;
    for (const auto& it : items) tot_bands += it.nbands;
    StageScope ts_(sizeof(T) == 8 ? MB_STAGE_LOCAL : MB_STAGE_LOCAL32, s, tot_bands);
    hipLaunchKernelGGL(kern, dim3((unsigned)units), dim3(256), lds, s, args[0], (const LineArgs<TI, T>*)da,
                       (const int32_t*)db, (int)items.size());
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

template <typename TI, typename T>
mb_status lines_batch_by_size(const std::vector<BatchItem>& items, TableUploader& up, hipStream_t s) {
    const Problem* p0 = items[0].p;
    if (p0->N1 != p0->N2) return MB_ERR_INVALID_ARG;
    switch (p0->N1) {
        case 16: return lines_batch_impl<TI, T, 16, 16>(items, up, s);
        case 24: return lines_batch_impl<TI, T, 24, 24>(items, up, s);
        case 25: return lines_batch_impl<TI, T, 25, 25>(items, up, s);
        case 27: return lines_batch_impl<TI, T, 27, 27>(items, up, s);
        case 30: return lines_batch_impl<TI, T, 30, 30>(items, up, s);
        case 32: return lines_batch_impl<TI, T, 32, 32>(items, up, s);
        case 36: return lines_batch_impl<TI, T, 36, 36>(items, up, s);
        case 40: return lines_batch_impl<TI, T, 40, 40>(items, up, s);
        default: break;
    }
    if constexpr (sizeof(T) == 4) {
        switch (p0->N1) {
            case 45: return lines_batch_impl<TI, T, 45, 45>(items, up, s);
            case 48: return lines_batch_impl<TI, T, 48, 48>(items, up, s);
            case 50: return lines_batch_impl<TI, T, 50, 50>(items, up, s);
            case 54: return lines_batch_impl<TI, T, 54, 54>(items, up, s);
            case 60: return lines_batch_impl<TI, T, 60, 60>(items, up, s);
            case 64: return lines_batch_impl<TI, T, 64, 64>(items, up, s);
            default: break;
        }
    }
    return MB_ERR_INVALID_ARG;
}

}  // namespace

// Returns MB_OK if a line kernel handled the grid, MB_ERR_INVALID_ARG if the grid
// has no line kernel (the caller then uses the generic one).
mb_status launch_local_lines(Problem* p, int ik, const void* c, void* part, int nbands, int ld, int prec,
                             hipStream_t s, int budget_kb) {
    if (p->order != KORD) return MB_ERR_INVALID_ARG;
    if (prec == 0) return lines_by_size<double, double>(p, ik, c, part, nbands, ld, s, budget_kb);
    if (prec == 1) return lines_by_size<float, float>(p, ik, c, part, nbands, ld, s, budget_kb);
    return lines_by_size<double, float>(p, ik, c, part, nbands, ld, s, budget_kb);
}

}  // namespace mb

namespace mb {
// items must share the in-plane grid; prec as for launch_local_lines
mb_status launch_local_lines_batch(const std::vector<BatchItem>& items, int prec, TableUploader& up,
                                   hipStream_t s) {
    if (items.empty()) return MB_OK;
    if (prec == 0) return lines_batch_by_size<double, double>(items, up, s);
    if (prec == 1) return lines_batch_by_size<float, float>(items, up, s);
    return lines_batch_by_size<double, float>(items, up, s);
}
}  // namespace mb
