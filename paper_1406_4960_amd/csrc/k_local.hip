// Local-potential part of H c: one workgroup per (band, knot interval) does, for
// each Gauss plane z_q of its interval,
//   evaluate   psi(G, z_q) = sum_t B_{s-1+t}(z_q) c(G, s-1+t)      (kappa terms)
//   scatter    psi(G) onto the in-plane grid (zero elsewhere)
//   inverse 2D FFT (unnormalised, exp(+i G.rho)), only grid rows that hold G
//   multiply   by V(rho, z_q) (real)
//   forward 2D FFT, exp(-i G.rho) / (N1 N2), gather the sphere
//   project    part(t, G) += w_q B_{s-1+t}(z_q) (V psi)(G, z_q)
// with the plane resident in LDS throughout.  Each interval's kappa partial rows
// are written once; the combine kernel adds the (up to kappa) partials of each
// spline row without atomics.  These are the matrix elements of a local
// potential in the mixed basis (Sec. II.B.1) with the in-plane transform taken
// on the grid (circular convolution), applied without forming the matrix.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "cplx.h"
#include "fft_lds.h"
#include "mbks_internal.h"

namespace mb {

namespace {

constexpr int KORD = 4;

template <typename TI, typename T>
struct LocalArgs {
    const cx<TI>* c;
    cx<T>* part;
    const T* bval;
    const T* wbval;
    const T* V;
    const int32_t* gmap;
    const int32_t* rows;
    const cx<T>* tw1;
    const cx<T>* tw2;
    int nbands, ld, ng, nint, nq, nb, N1, N2, nrows;
    T inv_n;
    FftPlan p1, p2;
};


// items == nullptr: one problem described by a0; otherwise a batch (item t owns work
// units [unit_begin[t], unit_begin[t+1]))
template <typename TI, typename T, int NT, int MAXG>
__global__ __launch_bounds__(NT) void k_local(LocalArgs<TI, T> a0, const LocalArgs<TI, T>* items,
                                              const int32_t* unit_begin, int nitems) {
    extern __shared__ unsigned char smem_raw[];
    unsigned L = xcd_logical(blockIdx.x, gridDim.x);
    LocalArgs<TI, T> a = a0;
    if (items) {
        const int it = batch_item_of(unit_begin, nitems, L);
        a = items[it];
        L -= (unsigned)unit_begin[it];
    }
    const int b = (int)(L % (unsigned)a.nbands);
    const int s = (int)(L / (unsigned)a.nbands);
    if (s >= a.nint) return;
    // the plane is stored with row stride N2 + 1 so that column passes (stride one
    // row) spread over the LDS banks
    cx<T>* grid = reinterpret_cast<cx<T>*>(smem_raw);
    const int npts = a.N1 * a.N2;
    const int P2 = a.N2 + 1;
    const int nstore = a.N1 * P2;
    cx<T>* tw1 = grid + nstore;
    cx<T>* tw2 = tw1 + a.N1;
    int32_t* rows = reinterpret_cast<int32_t*>(tw2 + a.N2);

    for (int e = threadIdx.x; e < a.N1; e += NT) tw1[e] = a.tw1[e];
    for (int e = threadIdx.x; e < a.N2; e += NT) tw2[e] = a.tw2[e];
    for (int e = threadIdx.x; e < a.nrows; e += NT) rows[e] = a.rows[e];

    const cx<TI>* cb = a.c + (size_t)b * a.nb * a.ld;
    cx<T> acc[KORD][MAXG];
#pragma unroll
    for (int t = 0; t < KORD; ++t)
#pragma unroll
        for (int k = 0; k < MAXG; ++k) acc[t][k] = mk<T>(0, 0);

    for (int jq = 0; jq < a.nq; ++jq) {
        const int q = s * a.nq + jq;
        for (int e = threadIdx.x; e < nstore; e += NT) grid[e] = mk<T>(0, 0);
        __syncthreads();
        T bv[KORD];
#pragma unroll
        for (int t = 0; t < KORD; ++t) bv[t] = a.bval[q * KORD + t];
#pragma unroll
        for (int k = 0; k < MAXG; ++k) {
            int g = threadIdx.x + k * NT;
            if (g < a.ng) {
                cx<T> psi = mk<T>(0, 0);
#pragma unroll
                for (int t = 0; t < KORD; ++t) {
                    int row = s - 1 + t;
                    if (row >= 0 && row < a.nb) {
                        cx<TI> cv = cb[(size_t)row * a.ld + g];
                        psi.x = fma(bv[t], (T)cv.x, psi.x);
                        psi.y = fma(bv[t], (T)cv.y, psi.y);
                    }
                }
                const int gm = a.gmap[g];
                grid[(gm / a.N2) * P2 + gm % a.N2] = psi;
            }
        }
        __syncthreads();
        // inverse transform: rows (axis 2) that hold G, then all columns (axis 1)
        fft_axis<T, NT>(grid, tw2, a.p2, a.nrows, rows, P2, 1, +1);
        fft_axis<T, NT>(grid, tw1, a.p1, a.N2, nullptr, 1, P2, +1);
        const T* Vq = a.V + (size_t)q * npts;
        for (int e = threadIdx.x; e < npts; e += NT) {
            const T v = Vq[e];
            const int o = (e / a.N2) * P2 + e % a.N2;
            const cx<T> u = grid[o];
            grid[o] = mk<T>(u.x * v, u.y * v);
        }
        __syncthreads();
        // forward transform: all columns, then the rows that hold G
        fft_axis<T, NT>(grid, tw1, a.p1, a.N2, nullptr, 1, P2, -1);
        fft_axis<T, NT>(grid, tw2, a.p2, a.nrows, rows, P2, 1, -1);
        T wb[KORD];
#pragma unroll
        for (int t = 0; t < KORD; ++t) wb[t] = a.wbval[q * KORD + t] * a.inv_n;
#pragma unroll
        for (int k = 0; k < MAXG; ++k) {
            int g = threadIdx.x + k * NT;
            if (g < a.ng) {
                const int gm = a.gmap[g];
                const cx<T> u = grid[(gm / a.N2) * P2 + gm % a.N2];
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
        int g = threadIdx.x + k * NT;
        if (g < a.ng) {
#pragma unroll
            for (int t = 0; t < KORD; ++t) pb[(size_t)t * a.ld + g] = acc[t][k];
        }
    }
}

template <typename TI, typename T, int NT, int MAXG>
mb_status run_local(const LocalArgs<TI, T>& a, size_t lds, hipStream_t s) {
    auto kern = k_local<TI, T, NT, MAXG>;
    if (lds > 65536)
        MB_HIP_TRY(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    unsigned nblocks = (unsigned)a.nbands * (unsigned)a.nint;
    StageScope ts_(sizeof(T) == 8 ? MB_STAGE_LOCAL : MB_STAGE_LOCAL32, s, a.nbands);
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(NT), lds, s, a, (const LocalArgs<TI, T>*)nullptr,
                       (const int32_t*)nullptr, 0);
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

template <typename TI, typename T>
LocalArgs<TI, T> make_local_args(Problem* p, int ik, const void* c, void* part, int nbands, int ld);

template <typename TI, typename T, int NT, int MAXG>
mb_status run_local_batch(const std::vector<LocalArgs<TI, T>>& args, const std::vector<int32_t>& begin, int units,
                          size_t lds, int64_t tot_bands, TableUploader& up, hipStream_t s) {
    void *ha, *da, *hb, *db;
    if (!up.reserve(args.size() * sizeof(args[0]), &ha, &da) || !up.reserve(begin.size() * 4, &hb, &db))
        return set_error(MB_ERR_OOM, "batch descriptor table full");
    std::memcpy(ha, args.data(), args.size() * sizeof(args[0]));
    std::memcpy(hb, begin.data(), begin.size() * 4);
    MB_HIP_TRY(hipMemcpyAsync(da, ha, args.size() * sizeof(args[0]), hipMemcpyHostToDevice, s));
    MB_HIP_TRY(hipMemcpyAsync(db, hb, begin.size() * 4, hipMemcpyHostToDevice, s));
    auto kern = k_local<TI, T, NT, MAXG>;
    if (lds > 65536)
        MB_HIP_TRY(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    StageScope ts_(sizeof(T) == 8 ? MB_STAGE_LOCAL : MB_STAGE_LOCAL32, s, tot_bands);
    hipLaunchKernelGGL(kern, dim3((unsigned)units), dim3(NT), lds, s, args[0], (const LocalArgs<TI, T>*)da,
                       (const int32_t*)db, (int)args.size());
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

// kernel variant (threads, G values per thread) that the single-problem launch uses
inline int local_variant(int work, int ng) {
    if (work <= 256 * MAXB && ng <= 256 * 2) return 0;
    if (work <= 256 * MAXB && ng <= 256 * 4) return 1;
    if (work <= 512 * MAXB && ng <= 512 * 4) return 2;
    if (work <= 1024 * MAXB && ng <= 1024 * 4) return 3;
    if (work <= 1024 * MAXB && ng <= 1024 * 8) return 4;
    return -1;
}

// one launch per kernel variant over the items that need it
template <typename TI, typename T>
mb_status local_batch_impl(const std::vector<BatchItem>& items, TableUploader& up, hipStream_t s) {
    std::vector<LocalArgs<TI, T>> args[5];
    std::vector<int32_t> begin[5];
    size_t lds[5] = {0, 0, 0, 0, 0};
    int units[5] = {0, 0, 0, 0, 0};
    int64_t bands[5] = {0, 0, 0, 0, 0};
    for (const auto& it : items) {
        if (it.p->order != KORD) return MB_ERR_INVALID_ARG;
        if (it.nbands == 0) continue;
        LocalArgs<TI, T> a = make_local_args<TI, T>(it.p, it.ik, it.c, it.part, it.nbands, it.ld);
        size_t l = sizeof(cx<T>) * ((size_t)a.N1 * (a.N2 + 1) + a.N1 + a.N2) + sizeof(int32_t) * a.nrows;
        if (l > 163840) return set_error(MB_ERR_INVALID_ARG, "in-plane grid does not fit in LDS");
        const int work = std::max(max_stage_work(a.p2, a.nrows), max_stage_work(a.p1, a.N2));
        const int v = local_variant(work, a.ng);
        if (v < 0) return set_error(MB_ERR_INVALID_ARG, "in-plane grid or G set too large for the local kernel");
        lds[v] = std::max(lds[v], l);
        args[v].push_back(a);
        begin[v].push_back(units[v]);
        units[v] += it.nbands * a.nint;
        bands[v] += it.nbands;
    }
    mb_status st = MB_OK;
    if (units[0] && st == MB_OK) st = run_local_batch<TI, T, 256, 2>(args[0], begin[0], units[0], lds[0], bands[0], up, s);
    if (units[1] && st == MB_OK) st = run_local_batch<TI, T, 256, 4>(args[1], begin[1], units[1], lds[1], bands[1], up, s);
    if (units[2] && st == MB_OK) st = run_local_batch<TI, T, 512, 4>(args[2], begin[2], units[2], lds[2], bands[2], up, s);
    if (units[3] && st == MB_OK) st = run_local_batch<TI, T, 1024, 4>(args[3], begin[3], units[3], lds[3], bands[3], up, s);
    if (units[4] && st == MB_OK) st = run_local_batch<TI, T, 1024, 8>(args[4], begin[4], units[4], lds[4], bands[4], up, s);
    return st;
}

template <typename TI, typename T>
LocalArgs<TI, T> make_local_args(Problem* p, int ik, const void* c, void* part, int nbands, int ld) {
    const KPoint& kp = p->kp[ik];
    LocalArgs<TI, T> a;
    a.c = (const cx<TI>*)c;
    a.part = (cx<T>*)part;
    const bool dbl = sizeof(T) == 8;
    a.bval = (const T*)(dbl ? (const void*)p->d_bval : (const void*)p->d_bvalf);
    a.wbval = (const T*)(dbl ? (const void*)p->d_wbval : (const void*)p->d_wbvalf);
    a.V = (const T*)(dbl ? (const void*)p->d_V : (const void*)p->d_Vf);
    a.gmap = kp.d_gmap;
    a.rows = kp.d_rows;
    a.tw1 = (const cx<T>*)(dbl ? p->d_tw1 : p->d_tw1f);
    a.tw2 = (const cx<T>*)(dbl ? p->d_tw2 : p->d_tw2f);
    a.nbands = nbands;
    a.ld = ld;
    a.ng = kp.ng;
    a.nint = p->nint;
    a.nq = p->nq;
    a.nb = p->nb;
    a.N1 = p->N1;
    a.N2 = p->N2;
    a.nrows = (int)kp.rows.size();
    a.inv_n = (T)(1.0 / ((double)p->N1 * p->N2));
    a.p1 = p->plan1;
    a.p2 = p->plan2;
    return a;
}

template <typename TI, typename T>
mb_status local_impl(Problem* p, int ik, const void* c, void* part, int nbands, int ld, hipStream_t s) {
    const KPoint& kp = p->kp[ik];
    LocalArgs<TI, T> a = make_local_args<TI, T>(p, ik, c, part, nbands, ld);
    size_t lds = sizeof(cx<T>) * ((size_t)p->N1 * (p->N2 + 1) + p->N1 + p->N2) + sizeof(int32_t) * a.nrows;
    if (lds > 163840) return set_error(MB_ERR_INVALID_ARG, "in-plane grid does not fit in LDS");
    int work = std::max(max_stage_work(p->plan2, a.nrows), max_stage_work(p->plan1, p->N2));
    // smallest block that covers the FFT stages and the G set
    switch (local_variant(work, kp.ng)) {
        case 0: return run_local<TI, T, 256, 2>(a, lds, s);
        case 1: return run_local<TI, T, 256, 4>(a, lds, s);
        case 2: return run_local<TI, T, 512, 4>(a, lds, s);
        case 3: return run_local<TI, T, 1024, 4>(a, lds, s);
        case 4: return run_local<TI, T, 1024, 8>(a, lds, s);
        default: break;
    }
    return set_error(MB_ERR_INVALID_ARG, "in-plane grid or G set too large for the local kernel");
}

// V(rho_j, z_q) = sum_atoms sum_t A_t sum_L exp(-|r - R - L|^2 / w_t^2) on the grid.
struct VTerm {
    double X, Y, Z, A, inv_w2;
    int nimg;
};

__global__ void k_vgrid(double* V, float* Vf, const VTerm* terms, int nterms, int N1, int N2, int nzq,
                        const double* zq, double a1x, double a1y, double a2x, double a2y) {
    const int npts = N1 * N2;
    size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)npts * nzq) return;
    int q = (int)(idx / npts);
    int e = (int)(idx - (size_t)q * npts);
    int j1 = e / N2, j2 = e - j1 * N2;
    double f1 = (double)j1 / N1, f2 = (double)j2 / N2;
    double x = f1 * a1x + f2 * a2x, y = f1 * a1y + f2 * a2y, z = zq[q];
    double v = 0.0;
    for (int t = 0; t < nterms; ++t) {
        VTerm m = terms[t];
        double dz = z - m.Z;
        double ez = dz * dz * m.inv_w2;
        if (ez > 60.0) continue;
        double sum = 0.0;
        for (int n1 = -m.nimg; n1 <= m.nimg; ++n1)
            for (int n2 = -m.nimg; n2 <= m.nimg; ++n2) {
                double dx = x - m.X - n1 * a1x - n2 * a2x;
                double dy = y - m.Y - n1 * a1y - n2 * a2y;
                double r2 = (dx * dx + dy * dy) * m.inv_w2;
                if (r2 < 60.0) sum += exp(-r2);
            }
        v += m.A * exp(-ez) * sum;
    }
    V[idx] = v;
    Vf[idx] = (float)v;
}

}  // namespace

mb_status launch_local(Problem* p, int ik, const void* c, void* part, int nbands, int ld, int prec,
                       hipStream_t s) {
    if (p->order != KORD) return set_error(MB_ERR_INVALID_ARG, "GPU kernels support order 4 only");
    // line-per-thread kernel for small grids, two-step line kernel for larger ones, unless
    // mb_autotune measured another choice for this k-point and precision;
    // MBKS_LOCAL_KERNEL=generic forces the generic kernel (used to cross-check them)
    const KPoint::Tune& tn = p->kp[ik].tune[prec];
    const char* sel = getenv("MBKS_LOCAL_KERNEL");
    const bool generic_only = sel && std::string(sel) == "generic";
    if (!generic_only && tn.set && tn.kind == 0) {
        mb_status st = launch_local_lines(p, ik, c, part, nbands, ld, prec, s, tn.budget_kb);
        if (st != MB_ERR_INVALID_ARG) return st;
    } else if (!generic_only && tn.set && tn.kind == 1) {
        mb_status st = launch_local_split(p, ik, c, part, nbands, ld, prec, s);
        if (st != MB_ERR_INVALID_ARG) return st;
    } else if (!generic_only && !(tn.set && tn.kind == 2)) {
        mb_status st = launch_local_lines(p, ik, c, part, nbands, ld, prec, s);
        if (st != MB_ERR_INVALID_ARG) return st;
        st = launch_local_split(p, ik, c, part, nbands, ld, prec, s);
        if (st != MB_ERR_INVALID_ARG) return st;
    }
    if (prec == 0) return local_impl<double, double>(p, ik, c, part, nbands, ld, s);
    if (prec == 1) return local_impl<float, float>(p, ik, c, part, nbands, ld, s);
    return local_impl<double, float>(p, ik, c, part, nbands, ld, s);
}

bool local_uses_planes(const Problem* p, int ik, int lp) {
    if (!plane_kernel_grid(p)) return false;
    // MBKS_LOCAL_KERNEL=generic or =split select the partial-row kernels (cross-checks)
    const char* sel = getenv("MBKS_LOCAL_KERNEL");
    if (sel && (std::string(sel) == "generic" || std::string(sel) == "split")) return false;
    const KPoint::Tune& tn = p->kp[ik].tune[lp];
    if (tn.set) return tn.kind == 3;
    // untuned: the plane kernel on the 128 x 64 grid, and in FP64 on the 36 x 36 grid
    // (graphene-like slab, 32 bands: H 0.23 against 0.26 ms with the line kernel; in FP32
    // the line kernel stays ahead, 0.072 against 0.080 ms local); elsewhere when
    // mb_autotune picks it
    return (p->N1 == 128 && p->N2 == 64) || (p->N1 == 36 && p->N2 == 36 && lp == 0);
}

mb_status launch_vgrid(Problem* p, hipStream_t s) {
    std::vector<VTerm> terms;
    double h1 = p->area / std::hypot(p->a2[0], p->a2[1]);
    double h2 = p->area / std::hypot(p->a1[0], p->a1[1]);
    double hmin = std::min(h1, h2);
    for (const auto& at : p->atoms) {
        const mb_species& sp = p->species[at.species];
        for (int t = 0; t < sp.ngauss; ++t) {
            VTerm m;
            m.X = at.pos[0];
            m.Y = at.pos[1];
            m.Z = at.pos[2];
            m.A = sp.gauss_A[t];
            m.inv_w2 = 1.0 / (sp.gauss_w[t] * sp.gauss_w[t]);
            // images closer than sqrt(60) w (exp(-60) ~ 1e-26) to the cell
            m.nimg = (int)std::ceil(std::sqrt(60.0) * sp.gauss_w[t] / hmin) + 1;
            terms.push_back(m);
        }
    }
    size_t n = (size_t)p->nzq * p->N1 * p->N2;
    if (terms.empty()) {
        MB_HIP_TRY(hipMemsetAsync(p->d_V, 0, n * sizeof(double), s));
        MB_HIP_TRY(hipMemsetAsync(p->d_Vf, 0, n * sizeof(float), s));
        return MB_OK;
    }
    VTerm* d_terms = nullptr;
    double* d_zq = nullptr;
    MB_HIP_TRY(hipMalloc(&d_terms, terms.size() * sizeof(VTerm)));
    MB_HIP_TRY(hipMalloc(&d_zq, p->zq.size() * sizeof(double)));
    MB_HIP_TRY(hipMemcpy(d_terms, terms.data(), terms.size() * sizeof(VTerm), hipMemcpyHostToDevice));
    MB_HIP_TRY(hipMemcpy(d_zq, p->zq.data(), p->zq.size() * sizeof(double), hipMemcpyHostToDevice));
    unsigned nblk = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_vgrid, dim3(nblk), dim3(256), 0, s, p->d_V, p->d_Vf, d_terms, (int)terms.size(),
                       p->N1, p->N2, p->nzq, d_zq, p->a1[0], p->a1[1], p->a2[0], p->a2[1]);
    MB_HIP_TRY(hipGetLastError());
    MB_HIP_TRY(hipStreamSynchronize(s));
    MB_HIP_TRY(hipFree(d_terms));
    MB_HIP_TRY(hipFree(d_zq));
    return MB_OK;
}

}  // namespace mb

namespace mb {
mb_status launch_local_batch(const std::vector<BatchItem>& items, int prec, TableUploader& up, hipStream_t s) {
    if (items.empty()) return MB_OK;
    if (prec == 0) return local_batch_impl<double, double>(items, up, s);
    if (prec == 1) return local_batch_impl<float, float>(items, up, s);
    return local_batch_impl<double, float>(items, up, s);
}
}  // namespace mb
