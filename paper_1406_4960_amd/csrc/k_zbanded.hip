// Operators that are banded along z and diagonal in G (Sec. II.B.1):
//   overlap  S = I_G (x) S_z,   kinetic T = 1/2 (D_z + |k+G|^2 S_z) per G,
// both with bandwidth kappa - 1 = 3.  The combine kernel reads c once per
// (band, row chunk, G) and writes
//   y(G,i) = (T c)(G,i) + sum of the local partials of row i
//            + sum_p F_p(G) Z_p(i) E_p <beta_p|c>
// so the kinetic term, the projection of the local potential and the
// Kleinman-Bylander expansion leave in one pass; with augmentation charges the overlap
// output gains the ultrasoft term sum_p F_p(G) Z_p(i) q_p <beta_p|c> (Sec. II.B.2) in
// the same pass.  s_solve and the preconditioner are forward / back substitutions with
// banded Cholesky factors.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "cplx.h"
#include "mbks_internal.h"

namespace mb {

namespace {

constexpr int KORD = 4;
constexpr int CH = 4;  // rows per thread in the combine kernel
// banded solves launched with at most this many 64-thread blocks (about 4 waves per CU)
// keep 8 rows of loads in flight per thread, larger launches 4
constexpr int64_t SOLVE_SMALL_WAVES = 1024;

template <typename TI, typename T>
struct CombineArgs {
    const cx<TI>* c;
    const cx<T>* part;    // [b][s][t][ld] (kappa rows per interval), [b][q][ld] (planes) or null
    const T* wb;          // planes: w_q B_{s-1+t}(z_q) as [q][kappa]
    const cx<T>* proj;    // [b][np] (already times E_p) or null
    const cx<T>* projq;   // [b][np] (already times q_p) or null: ultrasoft term of sy
    const cx<T>* F;       // [np][ld]
    const T* Z;           // [np][nb]
    const int32_t* zwin;  // [np][2]
    cx<TI>* y;            // may be null
    cx<TI>* sy;           // may be null
    const double* sband;  // band of the sy product: S_z (or the identity: sy = c + ultrasoft term)
    const double* dband;
    const double* kg2;
    int nbands, ld, ng, nb, nint, np;
    int nq;      // Gauss points per interval
    int planes;  // part holds one row per Gauss plane
};

// One block per (group of BB bands, chunk of CH rows, 256 columns); items == nullptr:
// one problem described by a0, else a batch (item t owns blocks [unit_begin[t],
// unit_begin[t+1])).  With BB > 1 every F_p(G) and Z_p(i) loaded for the projector
// expansion serves BB bands (many projectors: the expansion dominates the pass).
// AUG: sy also takes the expansion of projq (ultrasoft overlap).
template <typename TI, typename T, int BB, bool AUG>
__global__ __launch_bounds__(256) void k_combine(CombineArgs<TI, T> a0, const CombineArgs<TI, T>* items,
                                                 const int32_t* unit_begin, int nitems) {
    unsigned L = blockIdx.x;
    CombineArgs<TI, T> a = a0;
    if (items) {
        const int it = batch_item_of(unit_begin, nitems, L);
        a = items[it];
        L -= (unsigned)unit_begin[it];
    }
    const unsigned ncol = (unsigned)(a.ld + 255) / 256;
    const int g = (int)(L % ncol) * 256 + threadIdx.x;
    const int row = (int)(L / ncol);
    const int nchunk = (a.nb + CH - 1) / CH;
    const int bgrp = row / nchunk;
    const int i0 = (row - bgrp * nchunk) * CH;
    const int b0 = bgrp * BB;
    if (g >= a.ld || b0 >= a.nbands) return;
    const int nbg = min(BB, a.nbands - b0);
    const int i1 = min(i0 + CH, a.nb);
    if (g >= a.ng) {
        for (int bb = 0; bb < nbg; ++bb) {
            const size_t vb = (size_t)(b0 + bb) * a.nb * a.ld;
            for (int i = i0; i < i1; ++i) {
                if (a.y) a.y[vb + (size_t)i * a.ld + g] = mk<TI>(0, 0);
                if (a.sy) a.sy[vb + (size_t)i * a.ld + g] = mk<TI>(0, 0);
            }
        }
        return;
    }
    // projector expansion of the chunk's rows, sum_p F_p(G) Z_p(i) P'_p(b): each
    // F_p(G) is loaded once for all CH rows and BB bands
    constexpr int BQ = AUG ? BB : 1, CQ = AUG ? CH : 1;
    cx<T> nl[BB][CH], nq[BQ][CQ];
#pragma unroll
    for (int bb = 0; bb < BB; ++bb)
#pragma unroll
        for (int r = 0; r < CH; ++r) nl[bb][r] = mk<T>(0, 0);
#pragma unroll
    for (int bb = 0; bb < BQ; ++bb)
#pragma unroll
        for (int r = 0; r < CQ; ++r) nq[bb][r] = mk<T>(0, 0);
    const bool doy = a.y && a.proj;
    const bool doq = AUG && a.sy && a.projq;
    if (doy || doq) {
        for (int p = 0; p < a.np; ++p) {
            const int lo = max(a.zwin[2 * p], i0), hi = min(a.zwin[2 * p + 1], i1 - 1);
            if (lo > hi) continue;
            const cx<T> f = a.F[(size_t)p * a.ld + g];
            const T* zp = a.Z + (size_t)p * a.nb;
            T z[CH];
#pragma unroll
            for (int r = 0; r < CH; ++r) {
                const int i = i0 + r;
                z[r] = (i >= lo && i <= hi) ? zp[i] : (T)0;
            }
#pragma unroll
            for (int bb = 0; bb < BB; ++bb) {
                if (bb < nbg && doy) {
                    const cx<T> fp = cmul(f, a.proj[(size_t)(b0 + bb) * a.np + p]);
#pragma unroll
                    for (int r = 0; r < CH; ++r) {
                        const int i = i0 + r;
                        if (i >= lo && i <= hi) {
                            nl[bb][r].x = fma(z[r], fp.x, nl[bb][r].x);
                            nl[bb][r].y = fma(z[r], fp.y, nl[bb][r].y);
                        }
                    }
                }
                if constexpr (AUG) {
                    if (bb < nbg && doq) {
                        const cx<T> fq = cmul(f, a.projq[(size_t)(b0 + bb) * a.np + p]);
#pragma unroll
                        for (int r = 0; r < CH; ++r) {
                            const int i = i0 + r;
                            if (i >= lo && i <= hi) {
                                nq[bb][r].x = fma(z[r], fq.x, nq[bb][r].x);
                                nq[bb][r].y = fma(z[r], fq.y, nq[bb][r].y);
                            }
                        }
                    }
                }
            }
        }
    }
    // local part of the chunk's rows.  Planes: y(G, i) += sum over the intervals s of
    // B_i's support and their Gauss points q of w_q B_i(z_q) u_q(G); each plane row is
    // loaded once for all rows of the chunk it serves
    cx<T> loc[BB][CH];
#pragma unroll
    for (int bb = 0; bb < BB; ++bb)
#pragma unroll
        for (int r = 0; r < CH; ++r) loc[bb][r] = mk<T>(0, 0);
    if (a.y && a.part && a.planes) {
        const int s_lo = max(i0 - 2, 0), s_hi = min(i1, a.nint - 1);  // intervals i - 2 .. i + 1
        for (int sv = s_lo; sv <= s_hi; ++sv) {
            for (int jq = 0; jq < a.nq; ++jq) {
                const int q = sv * a.nq + jq;
                T w[CH];
#pragma unroll
                for (int r = 0; r < CH; ++r) {
                    const int t = i0 + r + 1 - sv;  // spline s - 1 + t = i
                    w[r] = (t >= 0 && t < KORD && i0 + r < i1) ? a.wb[(size_t)q * KORD + t] : (T)0;
                }
#pragma unroll
                for (int bb = 0; bb < BB; ++bb) {
                    if (bb < nbg) {
                        const cx<T> v = a.part[((size_t)(b0 + bb) * a.nint * a.nq + q) * a.ld + g];
#pragma unroll
                        for (int r = 0; r < CH; ++r) {
                            loc[bb][r].x = fma(w[r], v.x, loc[bb][r].x);
                            loc[bb][r].y = fma(w[r], v.y, loc[bb][r].y);
                        }
                    }
                }
            }
        }
    }
    const double kk = a.y ? 0.5 * a.kg2[g] : 0.0;
#pragma unroll
    for (int bb = 0; bb < BB; ++bb) {
        if (bb >= nbg) break;
        const size_t vb = (size_t)(b0 + bb) * a.nb * a.ld;
        const cx<TI>* cb = a.c + vb + g;
        // sliding window of c rows i-3 .. i+3 in TI precision
        cx<TI> w[2 * KORD - 1];
#pragma unroll
        for (int d = 0; d < 2 * KORD - 1; ++d) {
            int j = i0 - (KORD - 1) + d;
            w[d] = (j >= 0 && j < a.nb) ? cb[(size_t)j * a.ld] : mk<TI>(0, 0);
        }
#pragma unroll
        for (int r = 0; r < CH; ++r) {
            const int i = i0 + r;
            if (i >= i1) break;
            // banded products with symmetric S_z, D_z
            double sr = 0, si = 0, tr = 0, ti = 0;
#pragma unroll
            for (int d = -(KORD - 1); d <= KORD - 1; ++d) {
                int j = i + d;
                if (j < 0 || j >= a.nb) continue;
                int lo = d >= 0 ? i : j;
                int dd = d >= 0 ? d : -d;
                double sv = a.sband[lo * KORD + dd];
                cx<TI> cv = w[d + KORD - 1];
                sr += sv * (double)cv.x;
                si += sv * (double)cv.y;
                if (a.y) {
                    double tv = 0.5 * a.dband[lo * KORD + dd];
                    tr += tv * (double)cv.x;
                    ti += tv * (double)cv.y;
                }
            }
            if (a.sy) {
                double qr = 0.0, qi = 0.0;
                if constexpr (AUG) {
                    qr = (double)nq[bb][r].x;
                    qi = (double)nq[bb][r].y;
                }
                a.sy[vb + (size_t)i * a.ld + g] = mk<TI>((TI)(sr + qr), (TI)(si + qi));
            }
            if (a.y) {
                double yr = tr + kk * sr, yi = ti + kk * si;
                if (a.part && a.planes) {
                    yr += (double)loc[bb][r].x;
                    yi += (double)loc[bb][r].y;
                } else if (a.part) {
                    T pr = 0, pi = 0;
#pragma unroll
                    for (int t = 0; t < KORD; ++t) {
                        int s = i + 1 - t;
                        if (s < 0 || s >= a.nint) continue;
                        cx<T> v = a.part[(((size_t)(b0 + bb) * a.nint + s) * KORD + t) * a.ld + g];
                        pr += v.x;
                        pi += v.y;
                    }
                    yr += (double)pr;
                    yi += (double)pi;
                }
                yr += (double)nl[bb][r].x;
                yi += (double)nl[bb][r].y;
                a.y[vb + (size_t)i * a.ld + g] = mk<TI>((TI)yr, (TI)yi);
            }
            // slide the window
#pragma unroll
            for (int d = 0; d < 2 * KORD - 2; ++d) w[d] = w[d + 1];
            int jn = i + KORD;
            w[2 * KORD - 2] = (jn < a.nb) ? cb[(size_t)jn * a.ld] : mk<TI>(0, 0);
        }
    }
}

// x = (L L^T)^{-1} r along i with a banded lower factor lf[i][d] = L[i][i-d]
// (shared: lf[i*4+d], per_g = 0; or per G: lf[(i*4+d)*ld + g], per_g = 1).
// The recurrence is sequential in i; the loads of each chunk of U rows are issued
// together ahead of the chunk's arithmetic so their latencies overlap.  r may
// equal x (rows are read before they are overwritten).
template <typename TI, int U = 4>
__device__ inline void band_solve(const cx<TI>* r, cx<TI>* x, const double* lf, int nb, int ld, int g,
                                  int per_g, double theta, const cx<TI>* sv) {
    auto L = [&](int row, int d) -> double {
        return per_g ? lf[((size_t)row * KORD + d) * ld + g] : lf[row * KORD + d];
    };
    // forward: L w = r   (r - theta * sv when sv != null)
    cx<double> h1 = mk<double>(0, 0), h2 = h1, h3 = h1;  // w_{i-1}, w_{i-2}, w_{i-3}
    for (int i0 = 0; i0 < nb; i0 += U) {
        double vr[U], vi[U], l0[U], l1[U], l2[U], l3[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u;
            if (i < nb) {
                const size_t o = (size_t)i * ld + g;
                const cx<TI> rv = r[o];
                vr[u] = (double)rv.x;
                vi[u] = (double)rv.y;
                if (sv) {
                    const cx<TI> sx = sv[o];
                    vr[u] -= theta * (double)sx.x;
                    vi[u] -= theta * (double)sx.y;
                }
                l0[u] = L(i, 0);
                l1[u] = i >= 1 ? L(i, 1) : 0.0;
                l2[u] = i >= 2 ? L(i, 2) : 0.0;
                l3[u] = i >= 3 ? L(i, 3) : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u;
            if (i < nb) {
                double ar = vr[u] - l1[u] * h1.x - l2[u] * h2.x - l3[u] * h3.x;
                double ai = vi[u] - l1[u] * h1.y - l2[u] * h2.y - l3[u] * h3.y;
                const double inv = 1.0 / l0[u];
                h3 = h2;
                h2 = h1;
                h1 = mk<double>(ar * inv, ai * inv);
                x[(size_t)i * ld + g] = mk<TI>((TI)h1.x, (TI)h1.y);
            }
        }
    }
    // back: L^T x = w
    h1 = mk<double>(0, 0);
    h2 = h1;
    h3 = h1;  // x_{i+1}, x_{i+2}, x_{i+3}
    for (int i0 = nb - 1; i0 >= 0; i0 -= U) {
        double vr[U], vi[U], l0[U], l1[U], l2[U], l3[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 - u;
            if (i >= 0) {
                const cx<TI> wv = x[(size_t)i * ld + g];
                vr[u] = (double)wv.x;
                vi[u] = (double)wv.y;
                l0[u] = L(i, 0);
                l1[u] = i + 1 < nb ? L(i + 1, 1) : 0.0;
                l2[u] = i + 2 < nb ? L(i + 2, 2) : 0.0;
                l3[u] = i + 3 < nb ? L(i + 3, 3) : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 - u;
            if (i >= 0) {
                double ar = vr[u] - l1[u] * h1.x - l2[u] * h2.x - l3[u] * h3.x;
                double ai = vi[u] - l1[u] * h1.y - l2[u] * h2.y - l3[u] * h3.y;
                const double inv = 1.0 / l0[u];
                h3 = h2;
                h2 = h1;
                h1 = mk<double>(ar * inv, ai * inv);
                x[(size_t)i * ld + g] = mk<TI>((TI)h1.x, (TI)h1.y);
            }
        }
    }
}

// U rows of loads in flight per thread: 8 for small launches (a few waves per CU, the
// solve is one chain of dependent rows per thread), 4 for large ones (occupancy)
template <typename TI, int U>
__global__ __launch_bounds__(64) void k_ssolve(const cx<TI>* r, cx<TI>* x, const double* lband, int nbands,
                                                int ng, int nb, int ld) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (g >= ld || b >= nbands) return;
    const size_t vb = (size_t)b * nb * ld;
    if (g >= ng) {
        for (int i = 0; i < nb; ++i) x[vb + (size_t)i * ld + g] = mk<TI>(0, 0);
        return;
    }
    band_solve<TI, U>(r + vb, x + vb, lband, nb, ld, g, 0, 0.0, nullptr);
}

// banded Cholesky of kin (1/2 D_z + 1/2 |k+G|^2 S_z) + shift S_z for every G
__global__ void k_prec_factor(double* pf, const double* sband, const double* dband, const double* kg2,
                              double kin, double shift, int ng, int nb, int ld, int* fail) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    const double sh = kin * 0.5 * kg2[g] + shift;
    auto M = [&](int i, int j) -> double {
        if (i > j) { int t = i; i = j; j = t; }
        return kin * 0.5 * dband[i * KORD + (j - i)] + sh * sband[i * KORD + (j - i)];
    };
    auto L = [&](int i, int j) -> double& { return pf[((size_t)i * KORD + (i - j)) * ld + g]; };
    for (int i = 0; i < nb; ++i) {
        int j0 = max(0, i - (KORD - 1));
        for (int j = j0; j <= i; ++j) {
            double sum = M(i, j);
            for (int k = max(j0, j - (KORD - 1)); k < j; ++k) sum -= L(i, k) * L(j, k);
            if (j == i) {
                if (!(sum > 0)) { atomicExch(fail, 1); sum = 1.0; }
                L(i, i) = sqrt(sum);
            } else {
                L(i, j) = sum / L(j, j);
            }
        }
        for (int d = i + 1; d < KORD; ++d) pf[((size_t)i * KORD + d) * ld + g] = 0.0;
    }
}

template <int U>
__global__ __launch_bounds__(64) void k_prec_apply(const cx<double>* h, const cx<double>* sv,
                                                    const double* theta, const int32_t* sel, cx<double>* x,
                                                    const double* pf, int nvec, int ng, int nb, int ld) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (g >= ld || j >= nvec) return;
    const int src = sel ? sel[j] : j;
    const size_t vo = (size_t)j * nb * ld, vi = (size_t)src * nb * ld;
    if (g >= ng) {
        for (int i = 0; i < nb; ++i) x[vo + (size_t)i * ld + g] = mk<double>(0, 0);
        return;
    }
    band_solve<double, U>(h + vi, x + vo, pf, nb, ld, g, 1, theta ? theta[j] : 0.0, sv ? sv + vi : nullptr);
}

template <typename TI, typename T>
CombineArgs<TI, T> make_combine_args(Problem* p, int ik, const void* c, const void* part, const void* proj,
                                     void* y, void* sy, int nbands, int ld, bool planes = false,
                                     const void* projq = nullptr, const double* sband = nullptr) {
    const KPoint& kp = p->kp[ik];
    CombineArgs<TI, T> a;
    const bool dbl = sizeof(T) == 8;
    a.c = (const cx<TI>*)c;
    a.part = (const cx<T>*)part;
    a.proj = (const cx<T>*)proj;
    a.projq = (const cx<T>*)projq;
    a.F = (const cx<T>*)(dbl ? kp.d_F64 : kp.d_F32);
    a.Z = (const T*)(dbl ? (const void*)p->d_Z : (const void*)p->d_Zf);
    a.zwin = p->d_zwin;
    a.y = (cx<TI>*)y;
    a.sy = (cx<TI>*)sy;
    a.sband = sband ? sband : p->d_sband;
    a.dband = p->d_dband;
    a.kg2 = kp.d_kg2;
    a.nbands = nbands;
    a.ld = ld;
    a.ng = kp.ng;
    a.nb = p->nb;
    a.nint = p->nint;
    a.np = p->np;
    a.nq = p->nq;
    a.planes = planes ? 1 : 0;
    a.wb = (const T*)(dbl ? (const void*)p->d_wbval : (const void*)p->d_wbvalf);
    if (p->np == 0) {
        a.proj = nullptr;
        a.projq = nullptr;
    }
    return a;
}

inline int64_t combine_blocks(int nb, int ld, int nbands, int bb = 1) {
    return (int64_t)((ld + 255) / 256) * ((nbands + bb - 1) / bb) * ((nb + CH - 1) / CH);
}

// bands per thread of the combine kernel: 4 when the projector expansion dominates
// the pass (many projectors), else 1 (more workgroups for small band counts)
constexpr int COMBINE_BB_NP = 64;

template <typename TI, typename T>
mb_status combine_impl(Problem* p, int ik, const void* c, const void* part, const void* proj, void* y,
                       void* sy, int nbands, int ld, hipStream_t s, bool planes = false, const void* projq = nullptr,
                       const double* sband = nullptr) {
    CombineArgs<TI, T> a = make_combine_args<TI, T>(p, ik, c, part, proj, y, sy, nbands, ld, planes, projq, sband);
    const bool aug = sy && a.projq;
    const int cls = sizeof(T) == 8 ? 0 : sizeof(TI) == 8 ? 2 : 1;
    const KPoint::Tune& tn = p->kp[ik].tune[cls];
    bool wide = ((y && a.proj) || aug) &&
                (tn.set && tn.combine_bb ? tn.combine_bb == 4 : p->np >= COMBINE_BB_NP);
    if (wide) {
        const char* e = getenv("MBKS_COMBINE_BB");  // "1": one band per thread (cross-checks)
        if (e && e[0] == '1' && e[1] == 0) wide = false;
    }
    const int64_t nblk = combine_blocks(p->nb, ld, nbands, wide ? 4 : 1);
    if (nblk == 0) return MB_OK;
    if (nblk > (int64_t)1 << 24) return set_error(MB_ERR_INVALID_ARG, "block too large for the combine kernel");
    StageScope ts_(y ? MB_STAGE_COMBINE : MB_STAGE_SPSI, s, nbands);
    if (aug && wide)
        hipLaunchKernelGGL((k_combine<TI, T, 4, true>), dim3((unsigned)nblk), dim3(256), 0, s, a, nullptr, nullptr, 0);
    else if (aug)
        hipLaunchKernelGGL((k_combine<TI, T, 1, true>), dim3((unsigned)nblk), dim3(256), 0, s, a, nullptr, nullptr, 0);
    else if (wide)
        hipLaunchKernelGGL((k_combine<TI, T, 4, false>), dim3((unsigned)nblk), dim3(256), 0, s, a, nullptr, nullptr, 0);
    else
        hipLaunchKernelGGL((k_combine<TI, T, 1, false>), dim3((unsigned)nblk), dim3(256), 0, s, a, nullptr, nullptr, 0);
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

template <typename TI, typename T>
mb_status combine_batch_impl(const std::vector<BatchItem>& items, TableUploader& up, hipStream_t s) {
    std::vector<CombineArgs<TI, T>> args;
    std::vector<int32_t> begin;
    int64_t units = 0, tot_bands = 0;
    for (const auto& it : items) {
        args.push_back(make_combine_args<TI, T>(it.p, it.ik, it.c, it.part, it.proj, it.y, nullptr, it.nbands,
                                                it.ld));
        begin.push_back((int32_t)units);
        units += combine_blocks(it.p->nb, it.ld, it.nbands);
        tot_bands += it.nbands;
    }
    if (units == 0) return MB_OK;
    if (units > (int64_t)1 << 24) return set_error(MB_ERR_INVALID_ARG, "batch too large for the combine kernel");
    void *ha, *da, *hb, *db;
    if (!up.reserve(args.size() * sizeof(args[0]), &ha, &da) || !up.reserve(begin.size() * 4, &hb, &db))
        return set_error(MB_ERR_OOM, "batch descriptor table full");
    std::memcpy(ha, args.data(), args.size() * sizeof(args[0]));
    std::memcpy(hb, begin.data(), begin.size() * 4);
    MB_HIP_TRY(hipMemcpyAsync(da, ha, args.size() * sizeof(args[0]), hipMemcpyHostToDevice, s));
    MB_HIP_TRY(hipMemcpyAsync(db, hb, begin.size() * 4, hipMemcpyHostToDevice, s));
    StageScope ts_(MB_STAGE_COMBINE, s, tot_bands);
    hipLaunchKernelGGL((k_combine<TI, T, 1, false>), dim3((unsigned)units), dim3(256), 0, s, args[0],
                       (const CombineArgs<TI, T>*)da, (const int32_t*)db, (int)args.size());
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

}  // namespace

// prec: 0 = FP64 (c128), 1 = FP32 (c64), 2 = c128 vectors with FP32 local / nonlocal parts
mb_status launch_combine(Problem* p, int ik, const void* c, const void* part, const void* proj, void* y,
                         void* sy, int nbands, int ld, int prec, hipStream_t s, bool planes, const void* projq,
                         const double* sband) {
    if (prec == 0)
        return combine_impl<double, double>(p, ik, c, part, proj, y, sy, nbands, ld, s, planes, projq, sband);
    if (prec == 1) return combine_impl<float, float>(p, ik, c, part, proj, y, sy, nbands, ld, s, planes, projq, sband);
    return combine_impl<double, float>(p, ik, c, part, proj, y, sy, nbands, ld, s, planes, projq, sband);
}

mb_status launch_combine_batch(const std::vector<BatchItem>& items, int prec, TableUploader& up, hipStream_t s) {
    if (items.empty()) return MB_OK;
    if (prec == 0) return combine_batch_impl<double, double>(items, up, s);
    if (prec == 1) return combine_batch_impl<float, float>(items, up, s);
    return combine_batch_impl<double, float>(items, up, s);
}

mb_status launch_spsi_banded(Problem* p, int ik, const void* c, void* y, int nbands, int ld, int prec,
                             hipStream_t s) {
    if (p->wire) return wire_spsi(p, ik, c, y, nbands, ld, prec, s);
    if (prec == 1) return combine_impl<float, float>(p, ik, c, nullptr, nullptr, nullptr, y, nbands, ld, s);
    return combine_impl<double, double>(p, ik, c, nullptr, nullptr, nullptr, y, nbands, ld, s);
}

mb_status launch_ssolve_banded(Problem* p, int ik, const void* r, void* x, int nbands, int ld, int prec,
                               hipStream_t s) {
    if (p->wire) return wire_ssolve(p, ik, r, x, nbands, ld, prec, s);
    const KPoint& kp = p->kp[ik];
    dim3 grid((ld + 63) / 64, nbands);
    StageScope ts_(MB_STAGE_SSOLVE, s, nbands);
    const bool small = (int64_t)grid.x * grid.y <= SOLVE_SMALL_WAVES;
    if (prec == 1) {
        auto kern = small ? k_ssolve<float, 8> : k_ssolve<float, 4>;
        hipLaunchKernelGGL(kern, grid, dim3(64), 0, s, (const cx<float>*)r, (cx<float>*)x, p->d_lband, nbands,
                           kp.ng, p->nb, ld);
    } else {
        auto kern = small ? k_ssolve<double, 8> : k_ssolve<double, 4>;
        hipLaunchKernelGGL(kern, grid, dim3(64), 0, s, (const cx<double>*)r, (cx<double>*)x, p->d_lband, nbands,
                           kp.ng, p->nb, ld);
    }
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

mb_status launch_prec_factor(Problem* p, int ik, double sigma, hipStream_t s) {
    if (p->wire) return wire_prec_factor(p, ik, sigma, s);
    KPoint& kp = p->kp[ik];
    if (kp.d_pfac && kp.pfac_sigma == sigma) return MB_OK;
    if (!kp.d_pfac) MB_HIP_TRY(hipMalloc(&kp.d_pfac, (size_t)p->nb * KORD * kp.ld * sizeof(double)));
    int* d_fail = nullptr;
    MB_HIP_TRY(hipMalloc(&d_fail, sizeof(int)));
    MB_HIP_TRY(hipMemsetAsync(d_fail, 0, sizeof(int), s));
    // sigma > 0: (T + sigma S)^{-1}; sigma <= 0: S^{-1} (the plain generalized Krylov operator)
    double kin = sigma > 0 ? 1.0 : 0.0, shift = sigma > 0 ? sigma : 1.0;
    hipLaunchKernelGGL(k_prec_factor, dim3((kp.ng + 127) / 128), dim3(128), 0, s, kp.d_pfac, p->d_sband,
                       p->d_dband, kp.d_kg2, kin, shift, kp.ng, p->nb, kp.ld, d_fail);
    MB_HIP_TRY(hipGetLastError());
    int fail = 0;
    MB_HIP_TRY(hipMemcpyAsync(&fail, d_fail, sizeof(int), hipMemcpyDeviceToHost, s));
    MB_HIP_TRY(hipStreamSynchronize(s));
    MB_HIP_TRY(hipFree(d_fail));
    if (fail) return set_error(MB_ERR_NOT_SPD, "preconditioner block not positive definite");
    kp.pfac_sigma = sigma;
    return MB_OK;
}

mb_status launch_prec_apply(Problem* p, int ik, const void* h, const void* sv, const double* theta,
                            const int32_t* sel, void* x, int nvec, int ld, hipStream_t s) {
    if (p->wire) return wire_prec_apply(p, ik, h, sv, theta, sel, x, nvec, ld, s);
    const KPoint& kp = p->kp[ik];
    if (!kp.d_pfac || ld != kp.ld) return set_error(MB_ERR_INVALID_ARG, "preconditioner not built for this ld");
    dim3 grid((ld + 63) / 64, nvec);
    StageScope ts_(MB_STAGE_PRECOND, s, nvec);
    auto kern = (int64_t)grid.x * grid.y <= SOLVE_SMALL_WAVES ? k_prec_apply<8> : k_prec_apply<4>;
    hipLaunchKernelGGL(kern, grid, dim3(64), 0, s, (const cx<double>*)h, (const cx<double>*)sv, theta,
                       sel, (cx<double>*)x, kp.d_pfac, nvec, kp.ng, p->nb, ld);
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

}  // namespace mb
