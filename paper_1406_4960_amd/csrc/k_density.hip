// Electron density and Hartree potential on the in-plane grid at the Gauss planes
// (Sec. II.B.1: the charge density, and the Coulomb potential in the (z, g) form built
// from the 2D transform of 1/r).
//   density:  rho(rho_j, z_q) += sum_b w_b |psi_b(rho_j, z_q)|^2 / A with
//             psi_b(rho_j, z_q) = sum_G e^{i G.rho_j} sum_t B_{s-1+t}(z_q) c_b(G, s-1+t)
//             (the unnormalised inverse 2D transform of the evaluated plane; e^{i k.rho}
//             has modulus one).  One workgroup owns one Gauss plane and runs over the
//             bands, holding the plane's accumulators in registers: no atomics, and the
//             bands are summed in a fixed order.
//   Hartree:  rho(z_q, g) = 1/(N1 N2) sum_j rho(rho_j, z_q) e^{i g.rho_j}   (one plane per
//             workgroup through LDS), then for every grid frequency g
//               V(z_q, g) = sum_q' w_q' rho(z_q', g) (2 pi/|g|) e^{-|g| |z_q - z_q'|}
//               V(z_q, 0) = -2 pi sum_q' w_q' rho(z_q', 0) |z_q - z_q'|
//             by recursions over the ordered Gauss points (O(N_q) per g: the kernel
//             factorises on each side of z_q), then V(rho_j, z_q) = sum_g V(z_q, g)
//             e^{-i g.rho_j} (real part).  |g| is the grid frequency's shortest alias.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <string>
#include <vector>

#include "cplx.h"
#include "fft_lds.h"
#include "mbks_internal.h"

namespace mb {

namespace {

constexpr int KORD = 4;
constexpr double kTwoPi = 6.283185307179586476925286766559;

template <typename TI>
struct DensArgs {
    const cx<TI>* c;
    const double* w;       // nbands
    double* rho;           // [q][N1 N2]
    const double* bval;    // [q][kappa]
    const int32_t* gmap;
    const int32_t* rows;
    const cx<double>* tw1;
    const cx<double>* tw2;
    int nbands, ld, ng, nb, nq, nzq, N1, N2, nrows;
    double inv_area;
    FftPlan p1, p2;
};

size_t plane_lds_bytes(const Problem* p, int nrows) {
    return sizeof(cx<double>) * ((size_t)p->N1 * (p->N2 + 1) + p->N1 + p->N2) + sizeof(int32_t) * (size_t)nrows;
}

template <typename TI, int NT, int MAXP>
__global__ __launch_bounds__(NT) void k_density(DensArgs<TI> a) {
    extern __shared__ unsigned char smem_raw[];
    const int q = (int)xcd_logical(blockIdx.x, gridDim.x);
    if (q >= a.nzq) return;
    const int s = q / a.nq;
    cx<double>* grid = reinterpret_cast<cx<double>*>(smem_raw);
    const int npts = a.N1 * a.N2;
    const int P2 = a.N2 + 1;
    const int nstore = a.N1 * P2;
    cx<double>* tw1 = grid + nstore;
    cx<double>* tw2 = tw1 + a.N1;
    int32_t* rows = reinterpret_cast<int32_t*>(tw2 + a.N2);
    for (int e = threadIdx.x; e < a.N1; e += NT) tw1[e] = a.tw1[e];
    for (int e = threadIdx.x; e < a.N2; e += NT) tw2[e] = a.tw2[e];
    for (int e = threadIdx.x; e < a.nrows; e += NT) rows[e] = a.rows[e];
    double bv[KORD];
#pragma unroll
    for (int t = 0; t < KORD; ++t) bv[t] = a.bval[q * KORD + t];
    double acc[MAXP];
#pragma unroll
    for (int k = 0; k < MAXP; ++k) acc[k] = 0.0;
    for (int b = 0; b < a.nbands; ++b) {
        for (int e = threadIdx.x; e < nstore; e += NT) grid[e] = mk<double>(0, 0);
        __syncthreads();
        const cx<TI>* cb = a.c + (size_t)b * a.nb * a.ld;
        for (int g = threadIdx.x; g < a.ng; g += NT) {
            cx<double> psi = mk<double>(0, 0);
#pragma unroll
            for (int t = 0; t < KORD; ++t) {
                const int row = s - 1 + t;
                if (row >= 0 && row < a.nb) {
                    const cx<TI> cv = cb[(size_t)row * a.ld + g];
                    psi.x = fma(bv[t], (double)cv.x, psi.x);
                    psi.y = fma(bv[t], (double)cv.y, psi.y);
                }
            }
            const int gm = a.gmap[g];
            grid[(gm / a.N2) * P2 + gm % a.N2] = psi;
        }
        __syncthreads();
        // inverse transform, e^{+i G.rho}: the rows that hold G, then all columns
        fft_axis<double, NT>(grid, tw2, a.p2, a.nrows, rows, P2, 1, +1);
        fft_axis<double, NT>(grid, tw1, a.p1, a.N2, nullptr, 1, P2, +1);
        const double wb = a.w[b] * a.inv_area;
#pragma unroll
        for (int k = 0; k < MAXP; ++k) {
            const int e = threadIdx.x + k * NT;
            if (e < npts) {
                const cx<double> v = grid[(e / a.N2) * P2 + e % a.N2];
                acc[k] = fma(wb, v.x * v.x + v.y * v.y, acc[k]);
            }
        }
        __syncthreads();
    }
    double* rq = a.rho + (size_t)q * npts;
#pragma unroll
    for (int k = 0; k < MAXP; ++k) {
        const int e = threadIdx.x + k * NT;
        if (e < npts) rq[e] += acc[k];
    }
}

struct PlaneFftArgs {
    const double* rin;      // forward: real input planes [q][N1 N2]
    cx<double>* cout;       // forward: complex output planes
    const cx<double>* cin;  // inverse: complex input planes
    double* rout;           // inverse: real part of the output planes
    const cx<double>* tw1;
    const cx<double>* tw2;
    int nzq, N1, N2;
    double scale;
    FftPlan p1, p2;
};

// forward (sign +1, scaled): rho(z_q, g) of a real plane; inverse (sign -1): real part of
// sum_g V(z_q, g) e^{-i g.rho}.  Every grid row is transformed.
template <int NT, bool FWD>
__global__ __launch_bounds__(NT) void k_plane_fft(PlaneFftArgs a) {
    extern __shared__ unsigned char smem_raw[];
    const int q = (int)xcd_logical(blockIdx.x, gridDim.x);
    if (q >= a.nzq) return;
    cx<double>* grid = reinterpret_cast<cx<double>*>(smem_raw);
    const int npts = a.N1 * a.N2;
    const int P2 = a.N2 + 1;
    cx<double>* tw1 = grid + a.N1 * P2;
    cx<double>* tw2 = tw1 + a.N1;
    for (int e = threadIdx.x; e < a.N1; e += NT) tw1[e] = a.tw1[e];
    for (int e = threadIdx.x; e < a.N2; e += NT) tw2[e] = a.tw2[e];
    const size_t off = (size_t)q * npts;
    for (int e = threadIdx.x; e < npts; e += NT) {
        const int o = (e / a.N2) * P2 + e % a.N2;
        grid[o] = FWD ? mk<double>(a.rin[off + e], 0.0) : a.cin[off + e];
    }
    __syncthreads();
    if (FWD) {
        fft_axis<double, NT>(grid, tw2, a.p2, a.N1, nullptr, P2, 1, +1);
        fft_axis<double, NT>(grid, tw1, a.p1, a.N2, nullptr, 1, P2, +1);
        for (int e = threadIdx.x; e < npts; e += NT)
            a.cout[off + e] = cscale(grid[(e / a.N2) * P2 + e % a.N2], a.scale);
    } else {
        fft_axis<double, NT>(grid, tw1, a.p1, a.N2, nullptr, 1, P2, -1);
        fft_axis<double, NT>(grid, tw2, a.p2, a.N1, nullptr, P2, 1, -1);
        for (int e = threadIdx.x; e < npts; e += NT) a.rout[off + e] = grid[(e / a.N2) * P2 + e % a.N2].x;
    }
}

// V(z_q, g) from rho(z_q, g) for one grid frequency per thread: the z sums of the
// (z, g) Coulomb kernel over the Gauss points (ordered in z), each side of z_q by a
// recursion; columns are read and written coalesced across the frequencies
__global__ __launch_bounds__(256) void k_zcoulomb(const cx<double>* rg, cx<double>* vg, const double* gnorm,
                                                  const double* zq, const double* wq, int nzq, int npts) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= npts) return;
    const double g = gnorm[e];
    if (g > 0.0) {
        // L_q = sum_{q' <= q} w rho e^{-g (z_q - z_q')}
        cx<double> L = mk<double>(0, 0);
        for (int q = 0; q < nzq; ++q) {
            if (q > 0) L = cscale(L, exp(-g * (zq[q] - zq[q - 1])));
            const cx<double> r = rg[(size_t)q * npts + e];
            L.x = fma(wq[q], r.x, L.x);
            L.y = fma(wq[q], r.y, L.y);
            vg[(size_t)q * npts + e] = L;
        }
        // R_q = sum_{q' > q} w rho e^{-g (z_q' - z_q)}; V = (2 pi / g)(L + R)
        const double f = kTwoPi / g;
        cx<double> R = mk<double>(0, 0);
        for (int q = nzq - 1; q >= 0; --q) {
            const cx<double> l = vg[(size_t)q * npts + e];
            vg[(size_t)q * npts + e] = mk<double>(f * (l.x + R.x), f * (l.y + R.y));
            if (q > 0) {
                const cx<double> r = rg[(size_t)q * npts + e];
                R = mk<double>(fma(wq[q], r.x, R.x), fma(wq[q], r.y, R.y));
                R = cscale(R, exp(-g * (zq[q] - zq[q - 1])));
            }
        }
    } else {
        // -2 pi sum w rho |z_q - z_q'| = -2 pi (z_q A_q - B_q + (B - B_q) - z_q (A - A_q)),
        // A_q, B_q: sums of w rho and w rho z' over q' <= q; A, B: over all q'
        cx<double> A = mk<double>(0, 0), B = mk<double>(0, 0);
        for (int q = 0; q < nzq; ++q) {
            const cx<double> r = rg[(size_t)q * npts + e];
            A = mk<double>(fma(wq[q], r.x, A.x), fma(wq[q], r.y, A.y));
            B = mk<double>(fma(wq[q] * zq[q], r.x, B.x), fma(wq[q] * zq[q], r.y, B.y));
        }
        cx<double> Aq = mk<double>(0, 0), Bq = mk<double>(0, 0);
        for (int q = 0; q < nzq; ++q) {
            const cx<double> r = rg[(size_t)q * npts + e];
            Aq = mk<double>(fma(wq[q], r.x, Aq.x), fma(wq[q], r.y, Aq.y));
            Bq = mk<double>(fma(wq[q] * zq[q], r.x, Bq.x), fma(wq[q] * zq[q], r.y, Bq.y));
            const double z = zq[q];
            const double vr = z * Aq.x - Bq.x + (B.x - Bq.x) - z * (A.x - Aq.x);
            const double vi = z * Aq.y - Bq.y + (B.y - Bq.y) - z * (A.y - Aq.y);
            vg[(size_t)q * npts + e] = mk<double>(-kTwoPi * vr, -kTwoPi * vi);
        }
    }
}

// threads per workgroup for plane work of `work` butterflies per stage and npts points
int plane_threads(int work) {
    for (int nt : {256, 512, 1024})
        if (work <= nt * MAXB) return nt;
    return 0;
}

template <int NT, bool FWD>
mb_status run_plane_fft(const PlaneFftArgs& a, size_t lds, hipStream_t s) {
    auto kern = k_plane_fft<NT, FWD>;
    if (lds > 65536)
        MB_HIP_TRY(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kern, dim3(a.nzq), dim3(NT), lds, s, a);
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

template <bool FWD>
mb_status plane_fft(const PlaneFftArgs& a, int nt, size_t lds, hipStream_t s) {
    if (nt == 256) return run_plane_fft<256, FWD>(a, lds, s);
    if (nt == 512) return run_plane_fft<512, FWD>(a, lds, s);
    return run_plane_fft<1024, FWD>(a, lds, s);
}

template <typename TI, int NT, int MAXP>
mb_status run_density(const DensArgs<TI>& a, size_t lds, hipStream_t s) {
    auto kern = k_density<TI, NT, MAXP>;
    if (lds > 65536)
        MB_HIP_TRY(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    StageScope ts_(MB_STAGE_DENSITY, s, a.nbands);
    hipLaunchKernelGGL(kern, dim3(a.nzq), dim3(NT), lds, s, a);
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

template <typename TI, int NT>
mb_status density_by_points(const DensArgs<TI>& a, size_t lds, hipStream_t s) {
    const int npts = a.N1 * a.N2;
    if (npts <= NT * 4) return run_density<TI, NT, 4>(a, lds, s);
    if (npts <= NT * 8) return run_density<TI, NT, 8>(a, lds, s);
    if (npts <= NT * 16) return run_density<TI, NT, 16>(a, lds, s);
    return set_error(MB_ERR_INVALID_ARG, "density: in-plane grid larger than 16 x the workgroup");
}

template <typename TI>
mb_status density_impl(Problem* p, int ik, const void* c, int nbands, int ld, const double* w, double* rho,
                       hipStream_t s) {
    const KPoint& kp = p->kp[ik];
    DensArgs<TI> a;
    a.c = (const cx<TI>*)c;
    a.w = w;
    a.rho = rho;
    a.bval = p->d_bval;
    a.gmap = kp.d_gmap;
    a.rows = kp.d_rows;
    a.tw1 = (const cx<double>*)p->d_tw1;
    a.tw2 = (const cx<double>*)p->d_tw2;
    a.nbands = nbands;
    a.ld = ld;
    a.ng = kp.ng;
    a.nb = p->nb;
    a.nq = p->nq;
    a.nzq = p->nzq;
    a.N1 = p->N1;
    a.N2 = p->N2;
    a.nrows = (int)kp.rows.size();
    a.inv_area = 1.0 / p->area;
    a.p1 = p->plan1;
    a.p2 = p->plan2;
    const size_t lds = plane_lds_bytes(p, a.nrows);
    if (lds > 163840) return set_error(MB_ERR_INVALID_ARG, "density: in-plane grid does not fit in LDS");
    const int work = std::max(max_stage_work(p->plan2, a.nrows), max_stage_work(p->plan1, p->N2));
    const int nt = plane_threads(work);
    if (nt == 256) return density_by_points<TI, 256>(a, lds, s);
    if (nt == 512) return density_by_points<TI, 512>(a, lds, s);
    if (nt == 1024) return density_by_points<TI, 1024>(a, lds, s);
    return set_error(MB_ERR_INVALID_ARG, "density: in-plane grid too large for the plane kernel");
}

// device tables of the Hartree step: z_q, w_q and the shortest-alias |g| of every grid
// frequency (host FP64, uploaded on first use)
mb_status ensure_hartree_tables(Problem* p) {
    if (p->d_gnorm) return MB_OK;
    const int N1 = p->N1, N2 = p->N2;
    std::vector<double> gn((size_t)N1 * N2);
    for (int j1 = 0; j1 < N1; ++j1)
        for (int j2 = 0; j2 < N2; ++j2) {
            double best = -1.0;
            for (int n1 = -1; n1 <= 1; ++n1)
                for (int n2 = -1; n2 <= 1; ++n2) {
                    const double m1 = j1 + n1 * N1, m2 = j2 + n2 * N2;
                    const double gx = m1 * p->b1[0] + m2 * p->b2[0], gy = m1 * p->b1[1] + m2 * p->b2[1];
                    const double nrm = std::sqrt(gx * gx + gy * gy);
                    if (best < 0.0 || nrm < best - 1e-12) best = nrm;
                }
            gn[(size_t)j1 * N2 + j2] = best;
        }
    gn[0] = 0.0;
    double* d = nullptr;
    MB_HIP_TRY(hipMalloc(&d, gn.size() * sizeof(double)));
    MB_HIP_TRY(hipMemcpy(d, gn.data(), gn.size() * sizeof(double), hipMemcpyHostToDevice));
    double *dz = nullptr, *dw = nullptr;
    MB_HIP_TRY(hipMalloc(&dz, p->zq.size() * sizeof(double)));
    MB_HIP_TRY(hipMalloc(&dw, p->wq.size() * sizeof(double)));
    MB_HIP_TRY(hipMemcpy(dz, p->zq.data(), p->zq.size() * sizeof(double), hipMemcpyHostToDevice));
    MB_HIP_TRY(hipMemcpy(dw, p->wq.data(), p->wq.size() * sizeof(double), hipMemcpyHostToDevice));
    p->d_zq = dz;
    p->d_wq = dw;
    p->d_gnorm = d;
    return MB_OK;
}

}  // namespace

mb_status launch_density(Problem* p, int ik, const void* c, int nbands, int ld, const double* w, double* rho,
                         int prec, hipStream_t s) {
    if (nbands == 0) return MB_OK;
    if (p->order != KORD) return set_error(MB_ERR_INVALID_ARG, "GPU kernels support order 4 only");
    // the 128 x 64 grid: lane-split transforms (MBKS_DENSITY_KERNEL=generic: LDS transforms)
    const char* sel = getenv("MBKS_DENSITY_KERNEL");
    if (!(sel && std::string(sel) == "generic")) {
        mb_status st = launch_density_plane(p, ik, c, nbands, ld, w, rho, prec, s);
        if (st != MB_ERR_INVALID_ARG) return st;
    }
    if (prec == 0) return density_impl<double>(p, ik, c, nbands, ld, w, rho, s);
    return density_impl<float>(p, ik, c, nbands, ld, w, rho, s);
}

size_t hartree_work_bytes(const Problem* p, bool with_vzg) {
    return (with_vzg ? 1 : 2) * (size_t)p->nzq * p->N1 * p->N2 * sizeof(cx<double>);
}

mb_status launch_hartree(Problem* p, const double* rho, double* vh, void* vzg, void* work, hipStream_t s) {
    {
        mb_status st = ensure_hartree_tables(p);
        if (st != MB_OK) return st;
    }
    const int npts = p->N1 * p->N2;
    cx<double>* rg = (cx<double>*)work;
    cx<double>* vg = vzg ? (cx<double>*)vzg : rg + (size_t)p->nzq * npts;
    PlaneFftArgs a{};
    a.tw1 = (const cx<double>*)p->d_tw1;
    a.tw2 = (const cx<double>*)p->d_tw2;
    a.nzq = p->nzq;
    a.N1 = p->N1;
    a.N2 = p->N2;
    a.p1 = p->plan1;
    a.p2 = p->plan2;
    const size_t lds = sizeof(cx<double>) * ((size_t)p->N1 * (p->N2 + 1) + p->N1 + p->N2);
    if (lds > 163840) return set_error(MB_ERR_INVALID_ARG, "hartree: in-plane grid does not fit in LDS");
    const int nt = plane_threads(std::max(max_stage_work(p->plan2, p->N1), max_stage_work(p->plan1, p->N2)));
    if (nt == 0) return set_error(MB_ERR_INVALID_ARG, "hartree: in-plane grid too large for the plane kernel");
    StageScope ts_(MB_STAGE_HARTREE, s, p->nzq);
    a.rin = rho;
    a.cout = rg;
    a.scale = 1.0 / ((double)npts);
    mb_status st = plane_fft<true>(a, nt, lds, s);
    if (st != MB_OK) return st;
    hipLaunchKernelGGL(k_zcoulomb, dim3((npts + 255) / 256), dim3(256), 0, s, (const cx<double>*)rg, vg, p->d_gnorm,
                       p->d_zq, p->d_wq, p->nzq, npts);
    MB_HIP_TRY(hipGetLastError());
    a.cin = vg;
    a.rout = vh;
    return plane_fft<false>(a, nt, lds, s);
}

}  // namespace mb
