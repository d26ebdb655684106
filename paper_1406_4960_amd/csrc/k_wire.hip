// The 1D-periodic form on the GPU (B-splines along x and z, plane waves along y; the
// extension at the end of Sec. II.B.2).  H c in three passes:
//   k_wire_nlproj  P_p = E_p sum_{G,i,j} conj(F_p(G) X_p(i) Z_p(j)) c(G,i,j), one
//                  workgroup per (band, projector), fixed-order reduction;
//   k_wire_local   one workgroup per (band, z Gauss point z_p), walking the x knot
//                  intervals in rounds: stage t_i(G) = sum_j B_j(z_p) c(G,i,j) in LDS,
//                  evaluate psi(x_q, z_p, G) = sum_i B_i(x_q) t_i(G) on every FFT line of
//                  the round (lane-split ny-point lines), inverse transform, multiply by
//                  V(x_q, y, z_p) / ny, forward transform, gather, and project on the x
//                  splines, F(i, z_p, G) = sum_q w_q B_i(x_q) (V psi)(x_q, z_p, G); the
//                  rows shared with the next round carry over in LDS, so every F row is
//                  written once, complete (no atomics);
//   k_wire_combine y(G,i,j) = sum_p w_p B_j(z_p) F(i, z_p, G) + T c + sum_p F_p X_p Z_p P_p,
//                  the banded kinetic and overlap sums in FP64, one thread per (band, i, G)
//                  and chunk of 4 z rows.
// S^{-1} = S_x^{-1} (x) S_z^{-1}: two banded Cholesky substitutions.  The eigensolver's
// preconditioner (T + sigma S)^{-1} diagonalises the z direction (D_z u = lambda S_z u,
// u S_z-orthonormal): per z eigenvector j' and G it is the banded x problem
// 1/2 D_x + (lambda_j' / 2 + |k+G|^2 / 2 + sigma) S_x, so it runs as a dense z
// transform, banded x substitutions and the back transform.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <string>
#include <vector>

#include "cplx.h"
#include "fft_line.h"
#include "lane_fft.h"
#include "mbks_internal.h"

namespace mb {

namespace {

constexpr int KORD = 4;
constexpr int WNT = 256;  // threads of the local, projection and transform kernels
using fftl::line_fft;

template <typename T>
mb_status put(T** dst, const std::vector<T>& src) {
    if (src.empty()) {
        *dst = nullptr;
        return MB_OK;
    }
    if (hipMalloc(dst, src.size() * sizeof(T)) != hipSuccess) return set_error(MB_ERR_OOM, "hipMalloc failed");
    MB_HIP_TRY(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return MB_OK;
}

mb_status putf(float** dst, const std::vector<double>& src) { return put(dst, std::vector<float>(src.begin(), src.end())); }

template <typename T>
__device__ __forceinline__ void rfma(cx<T>& acc, T w, cx<T> v) {
    acc.x = fma(w, v.x, acc.x);
    acc.y = fma(w, v.y, acc.y);
}

// ---- potential on the Gauss points ------------------------------------------------------
struct WTerm {
    double A, w, X, Y, Z;
    int nimg;
};

// V[p][q][n] = sum_terms A exp(-((x_q - X)^2 + (z_p - Z)^2) / w^2) sum_images exp(-(y_n - Y - m L)^2 / w^2),
// divided by ny (the scale of the forward transform)
__global__ void k_wire_vgrid(double* V, float* Vf, const double* xq, const double* zq, const WTerm* terms,
                             int nterm, int nxq, int nzq, int ny, double L) {
    const size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n_all = (size_t)nzq * nxq * ny;
    if (o >= n_all) return;
    const int n = (int)(o % ny);
    const int q = (int)((o / ny) % nxq);
    const int p = (int)(o / ((size_t)ny * nxq));
    const double x = xq[q], z = zq[p], y = n * L / ny;
    double v = 0.0;
    for (int t = 0; t < nterm; ++t) {
        const WTerm tm = terms[t];
        const double iw2 = 1.0 / (tm.w * tm.w);
        double fy = 0.0;
        for (int m = -tm.nimg; m <= tm.nimg; ++m) {
            const double dy = y - tm.Y - m * L;
            fy += exp(-dy * dy * iw2);
        }
        const double dx = x - tm.X, dz = z - tm.Z;
        v += tm.A * exp(-(dx * dx + dz * dz) * iw2) * fy;
    }
    v /= ny;
    V[o] = v;
    Vf[o] = (float)v;
}

// ---- local potential ----------------------------------------------------------------------
template <typename TI, typename T>
struct WLocalArgs {
    const cx<TI>* c;       // [b][i][j][ld]
    cx<T>* F;              // [b][i][p][ld]
    const T* bx;           // [q][kappa] spline values along x
    const T* wbx;          // [q][kappa] w_q times them
    const T* bz;           // [p][kappa]
    const T* V;            // [p][q][ny], V / ny
    const cx<T>* tw;       // [ny] exp(+2 pi i k / ny)
    const int32_t* gtab;   // [ny] G index at each y-grid position, -1 none
    int nbands, ld, ng, nbx, nbz, nintx, nq, nxq, nzq;
};

template <typename T, int NY>
constexpr size_t wire_hdr() {
    return ((sizeof(cx<T>) * NY + sizeof(int32_t) * NY + 255) / 256) * 256;
}

template <typename T, int NY, int Q, int NT>
size_t wire_local_lds(int ng, int nq) {
    const int LR = NT / Q, RI = LR / nq, NR = RI + 3;
    return wire_hdr<T, NY>() + sizeof(cx<T>) * (size_t)ng * (2 * NR + LR);
}

template <typename TI, typename T, int NY, int Q, int NT>
__global__ __launch_bounds__(NT) void k_wire_local(WLocalArgs<TI, T> a) {
    constexpr int L = NY / Q;
    constexpr int LR = NT / Q;  // lines per round
    extern __shared__ unsigned char smem_raw[];
    const int RI = LR / a.nq;    // knot intervals per round (host checks >= 1)
    const int NR = RI + 3;       // spline rows a round touches
    cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
    int32_t* gt = reinterpret_cast<int32_t*>(tw + NY);
    cx<T>* tb = reinterpret_cast<cx<T>*>(smem_raw + wire_hdr<T, NY>());
    cx<T>* ub = tb + (size_t)NR * a.ng;
    cx<T>* acc = ub + (size_t)LR * a.ng;

    // work order: the bands of one z Gauss point are consecutive logical workgroups, which
    // share an XCD and its L2 (the point's potential slab and coefficient rows)
    const unsigned lw = xcd_logical(blockIdx.x, gridDim.x);
    const int b = (int)(lw % (unsigned)a.nbands);
    const int p = (int)(lw / (unsigned)a.nbands);
    if (p >= a.nzq) return;
    const int e = p / a.nq;  // z knot interval of the point
    const int tid = threadIdx.x;
    for (int k = tid; k < NY; k += NT) {
        tw[k] = a.tw[k];
        gt[k] = a.gtab[k];
    }
    for (int o = tid; o < NR * a.ng; o += NT) acc[o] = mk<T>(0, 0);
    T bzv[KORD];
#pragma unroll
    for (int t = 0; t < KORD; ++t) bzv[t] = a.bz[(size_t)p * KORD + t];
    const cx<TI>* cb = a.c + (size_t)b * a.nbx * a.nbz * a.ld;
    cx<T>* Fb = a.F + (size_t)b * a.nbx * a.nzq * a.ld;
    // line and lane of this thread (a line's Q lanes sit in one 16-lane row)
    const int line = (tid >> 4) * (16 / Q) + LaneMap<Q>::line(tid & 15);
    const int l = LaneMap<Q>::lane(tid & 15);
    __syncthreads();

    for (int r0 = 0; r0 < a.nintx; r0 += RI) {
        const int r1 = min(r0 + RI, a.nintx);
        const int nrow = r1 - r0 + 3;  // spline rows r0 - 1 .. r1 + 1
        // z contraction of the rows this round needs
        for (int o = tid; o < nrow * a.ng; o += NT) {
            const int rl = o / a.ng, g = o - rl * a.ng;
            const int i = r0 - 1 + rl;
            cx<T> v = mk<T>(0, 0);
            if (i >= 0 && i < a.nbx) {
#pragma unroll
                for (int t = 0; t < KORD; ++t) {
                    const int j = e - 1 + t;
                    if (j < 0 || j >= a.nbz) continue;
                    const cx<TI> cv = cb[((size_t)i * a.nbz + j) * a.ld + g];
                    rfma(v, bzv[t], mk<T>((T)cv.x, (T)cv.y));
                }
            }
            tb[o] = v;
        }
        __syncthreads();

        // one FFT line per x Gauss point of the round (whole lines active or idle)
        const int nl = (r1 - r0) * a.nq;
        if (line < nl) {
            const int xq = r0 * a.nq + line;
            const int s = xq / a.nq;
            T bxv[KORD];
#pragma unroll
            for (int t = 0; t < KORD; ++t) bxv[t] = a.bx[(size_t)xq * KORD + t];
            const cx<T>* trow = tb + (size_t)(s - r0) * a.ng;
            cx<T> x[L];
#pragma unroll
            for (int m = 0; m < L; ++m) {
                const int gi = gt[l + Q * m];
                cx<T> v = mk<T>(0, 0);
                if (gi >= 0) {
#pragma unroll
                    for (int t = 0; t < KORD; ++t) rfma(v, bxv[t], trow[(size_t)t * a.ng + gi]);
                }
                x[m] = v;
            }
            line_fft<T, L, +1>(x);
#pragma unroll
            for (int k = 1; k < L; ++k) x[k] = cmul(x[k], tw_at<T, +1>(tw, l * k));
            dif_lanes<T, L, Q, NY, +1>(x, l, tw);
            const T* vp = a.V + ((size_t)p * a.nxq + xq) * NY + L * bitrev_lane<Q>(l);
#pragma unroll
            for (int k = 0; k < L; ++k) {
                const T v = vp[k];
                x[k] = mk<T>(x[k].x * v, x[k].y * v);
            }
            dit_lanes<T, L, Q, NY, -1>(x, l, tw);
#pragma unroll
            for (int k = 1; k < L; ++k) x[k] = cmul(x[k], tw_at<T, -1>(tw, l * k));
            line_fft<T, L, -1>(x);
#pragma unroll
            for (int m = 0; m < L; ++m) {
                const int gi = gt[l + Q * m];
                if (gi >= 0) ub[(size_t)line * a.ng + gi] = x[m];
            }
        }
        __syncthreads();

        // x projection onto the spline rows of the round
        for (int o = tid; o < nrow * a.ng; o += NT) {
            const int rl = o / a.ng, g = o - rl * a.ng;
            const int i = r0 - 1 + rl;
            cx<T> v = acc[o];
            const int s0 = max(i - 2, r0), s1 = min(i + 1, r1 - 1);
            for (int s = s0; s <= s1; ++s) {
                const int t = i - s + 1;
                for (int jq = 0; jq < a.nq; ++jq) {
                    const int xq = s * a.nq + jq;
                    rfma(v, a.wbx[(size_t)xq * KORD + t], ub[(size_t)((s - r0) * a.nq + jq) * a.ng + g]);
                }
            }
            acc[o] = v;
        }
        __syncthreads();
        // rows below r1 - 1 are complete (the next interval starts at row r1 - 1)
        const bool last = r1 >= a.nintx;
        const int ndone = last ? nrow : nrow - 3;
        for (int o = tid; o < ndone * a.ng; o += NT) {
            const int rl = o / a.ng, g = o - rl * a.ng;
            const int i = r0 - 1 + rl;
            if (i >= 0 && i < a.nbx) Fb[((size_t)i * a.nzq + p) * a.ld + g] = acc[o];
        }
        if (last) break;
        __syncthreads();
        // carry the three open rows to the front (through tb, free until the next stage)
        for (int o = tid; o < 3 * a.ng; o += NT) tb[o] = acc[(size_t)(nrow - 3) * a.ng + o];
        __syncthreads();
        for (int o = tid; o < NR * a.ng; o += NT) acc[o] = o < 3 * a.ng ? tb[o] : mk<T>(0, 0);
        __syncthreads();
    }
}

template <typename TI, typename T, int NY, int Q, int NT>
mb_status wire_local_launch_nt(const WLocalArgs<TI, T>& a, hipStream_t s) {
    const size_t lds = wire_local_lds<T, NY, Q, NT>(a.ng, a.nq);
    if (lds > 160 * 1024) return set_error(MB_ERR_INVALID_ARG, "1D-periodic local kernel: plane-wave set too large for LDS");
    auto kern = k_wire_local<TI, T, NY, Q, NT>;
    if (lds > 64 * 1024) MB_HIP_TRY(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const size_t nwg = (size_t)a.nbands * a.nzq;
    if (nwg > 0x7fffffffull) return set_error(MB_ERR_INVALID_ARG, "1D-periodic local kernel: too many bands");
    hipLaunchKernelGGL(kern, dim3((unsigned)nwg), dim3(NT), lds, s, a);
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

// 512 threads per workgroup (MBKS_WIRE_LOCAL_THREADS=256 selects 256: half the lines per
// round, twice the rounds; measured on the 19-line ribbon, 96 bands: 6.5 against 7.2 ms in
// FP64, 3.5 against 3.7 ms in FP32)
template <typename TI, typename T, int NY, int Q>
mb_status wire_local_launch(const WLocalArgs<TI, T>& a, hipStream_t s) {
    const char* sel = getenv("MBKS_WIRE_LOCAL_THREADS");
    if (sel && std::string(sel) == "256") return wire_local_launch_nt<TI, T, NY, Q, 256>(a, s);
    return wire_local_launch_nt<TI, T, NY, Q, 512>(a, s);
}

template <typename TI, typename T>
mb_status wire_local_dispatch(const WLocalArgs<TI, T>& a, int ny, hipStream_t s) {
    switch (ny) {
        case 8: return wire_local_launch<TI, T, 8, 2>(a, s);
        case 12: return wire_local_launch<TI, T, 12, 4>(a, s);
        case 16: return wire_local_launch<TI, T, 16, 4>(a, s);
        case 24: return wire_local_launch<TI, T, 24, 8>(a, s);
        case 32: return wire_local_launch<TI, T, 32, 8>(a, s);
        case 48: return wire_local_launch<TI, T, 48, 8>(a, s);
        case 64: return wire_local_launch<TI, T, 64, 8>(a, s);
        case 128: return wire_local_launch<TI, T, 128, 16>(a, s);
        default: return set_error(MB_ERR_INVALID_ARG, "1D-periodic local kernel: unsupported ny");
    }
}

// ---- projections ------------------------------------------------------------------------
template <typename TI, typename T>
__global__ __launch_bounds__(WNT) void k_wire_nlproj(const cx<TI>* c, cx<T>* proj, const cx<T>* Fp, const T* X,
                                                     const T* Z, const T* E, const int32_t* xwin,
                                                     const int32_t* zwin, int nbands, int ld, int ng, int nbx,
                                                     int nbz, int np) {
    __shared__ cx<T> red[WNT];
    const int q = blockIdx.x, b = blockIdx.y;
    const int x0 = xwin[2 * q], x1 = xwin[2 * q + 1], z0 = zwin[2 * q], z1 = zwin[2 * q + 1];
    const int nx = x1 - x0 + 1, nz = z1 - z0 + 1;
    cx<T> acc = mk<T>(0, 0);
    if (nx > 0 && nz > 0) {
        const int64_t count = (int64_t)nx * nz * ng;
        const cx<TI>* cb = c + (size_t)b * nbx * nbz * ld;
        for (int64_t o = threadIdx.x; o < count; o += WNT) {
            const int g = (int)(o % ng);
            const int64_t r = o / ng;
            const int j = z0 + (int)(r % nz), i = x0 + (int)(r / nz);
            const cx<TI> cv = cb[((size_t)i * nbz + j) * ld + g];
            const T w = X[(size_t)q * nbx + i] * Z[(size_t)q * nbz + j];
            const cx<T> f = Fp[(size_t)q * ld + g];
            cx<T> t = mk<T>(0, 0);
            cfmac(t, f, mk<T>((T)cv.x, (T)cv.y));
            rfma(acc, w, t);
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = WNT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) proj[(size_t)b * np + q] = cscale(red[0], E[q]);
}

// ---- combine: z projection, kinetic, overlap, nonlocal expansion ----------------------------
template <typename TI, typename T>
struct WCombineArgs {
    const cx<TI>* c;
    const cx<T>* F;        // local x projections or null
    const cx<T>* proj;     // E-scaled projections [b][np] or null
    cx<TI>* y;
    cx<TI>* sy;            // S c or null
    const T* wbz;          // [p][kappa]
    const double *sx, *dx, *sz, *dz;
    const double* kg2;
    const cx<T>* Fp;
    const T* X;
    const T* Z;
    const int32_t* zwin;
    const int32_t* ploff;
    const int32_t* plist;
    int nbands, ld, ng, nbx, nbz, nintz, nq, nzq, np;
    int s_only;            // y = S c only
};

__device__ __forceinline__ double band_at(const double* m, int i, int i2) {
    const int lo = min(i, i2), d = abs(i - i2);
    return d < KORD ? m[lo * KORD + d] : 0.0;
}

// One thread per (band, x row i, G) and a chunk of WJB consecutive z rows j0 .. j0+WJB-1
// (the chunk is blockIdx.y, so the z band and spline coefficients are uniform over the
// workgroup): each coefficient row and each F row loaded serves every output of the chunk
// it touches (the kinetic stencil as z sums per x neighbour, then the x sum).
template <typename TI, typename T, int WJB>
__global__ __launch_bounds__(256) void k_wire_combine(WCombineArgs<TI, T> a) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int j0 = blockIdx.y * WJB;
    const int b = blockIdx.z;
    if (o >= (int64_t)a.nbx * a.ld) return;
    const int i = (int)(o / a.ld), g = (int)(o - (int64_t)i * a.ld);
    const int nj = min(WJB, a.nbz - j0);
    const size_t vb = (size_t)b * a.nbx * a.nbz * a.ld;
    const size_t ob = vb + ((size_t)i * a.nbz + j0) * a.ld + g;
    if (g >= a.ng) {
        for (int t = 0; t < nj; ++t) {
            a.y[ob + (size_t)t * a.ld] = mk<TI>(0, 0);
            if (a.sy) a.sy[ob + (size_t)t * a.ld] = mk<TI>(0, 0);
        }
        return;
    }
    const double k2 = a.s_only ? 0.0 : 0.5 * a.kg2[g];
    cx<double> kin[WJB], sc[WJB];
#pragma unroll
    for (int t = 0; t < WJB; ++t) kin[t] = sc[t] = mk<double>(0, 0);
    // Banded sums over x (i2 = i - 3 .. i + 3) and z (the chunk's rows +- 3).  Loads take
    // clamped, valid indices and out-of-range terms get zero coefficients, so that no
    // load sits under a branch (the compiler waits for every load in flight where
    // branches join, which serialized these loads)
    for (int di = -(KORD - 1); di <= KORD - 1; ++di) {
        const int i2r = i + di;
        const bool iok = i2r >= 0 && i2r < a.nbx;
        const int i2 = iok ? i2r : i;
        const int xlo = min(i, i2), xd = iok ? (di >= 0 ? di : -di) : 0;
        const double sx0 = a.sx[xlo * KORD + xd], dx0 = a.dx[xlo * KORD + xd];
        const double sxv = iok ? sx0 : 0.0, dxv = iok ? dx0 : 0.0;
        const cx<TI>* cr = a.c + vb + (size_t)i2 * a.nbz * a.ld + g;
        cx<TI> cv[WJB + 2 * (KORD - 1)];
#pragma unroll
        for (int u = 0; u < WJB + 2 * (KORD - 1); ++u) {
            const int jj = min(max(j0 - (KORD - 1) + u, 0), a.nbz - 1);
            cv[u] = cr[(size_t)jj * a.ld];
        }
        cx<double> az[WJB], dz[WJB];
#pragma unroll
        for (int t = 0; t < WJB; ++t) az[t] = dz[t] = mk<double>(0, 0);
#pragma unroll
        for (int u = 0; u < WJB + 2 * (KORD - 1); ++u) {
            const int jj = j0 - (KORD - 1) + u;
            const bool jok = jj >= 0 && jj < a.nbz;
            const double vr = (double)cv[u].x, vi = (double)cv[u].y;
#pragma unroll
            for (int t = 0; t < WJB; ++t) {
                const int dj = u - (KORD - 1) - t;
                if (dj < -(KORD - 1) || dj > KORD - 1) continue;  // compile-time
                const int j = j0 + t;
                const bool ok = jok && j < a.nbz;
                const int zlo = ok ? min(j, jj) : 0, zd = dj >= 0 ? dj : -dj;
                const double s0 = a.sz[zlo * KORD + zd], d0 = a.dz[zlo * KORD + zd];
                const double sv = ok ? s0 : 0.0, dv = ok ? d0 : 0.0;
                az[t].x = fma(sv, vr, az[t].x);
                az[t].y = fma(sv, vi, az[t].y);
                dz[t].x = fma(dv, vr, dz[t].x);
                dz[t].y = fma(dv, vi, dz[t].y);
            }
        }
        const double ka = 0.5 * dxv + k2 * sxv, kd = 0.5 * sxv;
#pragma unroll
        for (int t = 0; t < WJB; ++t) {
            kin[t].x = fma(ka, az[t].x, fma(kd, dz[t].x, kin[t].x));
            kin[t].y = fma(ka, az[t].y, fma(kd, dz[t].y, kin[t].y));
            sc[t].x = fma(sxv, az[t].x, sc[t].x);
            sc[t].y = fma(sxv, az[t].y, sc[t].y);
        }
    }
    if (a.s_only) {
#pragma unroll
        for (int t = 0; t < WJB; ++t)
            if (t < nj) a.y[ob + (size_t)t * a.ld] = mk<TI>((TI)sc[t].x, (TI)sc[t].y);
        return;
    }
    cx<T> v[WJB];
#pragma unroll
    for (int t = 0; t < WJB; ++t) v[t] = mk<T>(0, 0);
    if (a.F) {
        const cx<T>* Fr = a.F + ((size_t)b * a.nbx + i) * a.nzq * a.ld + g;
        // the Gauss points of the intervals meeting the chunk, as one flat range (the
        // interval index is uniform, so the loads of consecutive points overlap)
        const int p_lo = max(0, j0 - 2) * a.nq, p_hi = (min(a.nintz - 1, j0 + WJB) + 1) * a.nq;
#pragma unroll 5
        for (int p = p_lo; p < p_hi; ++p) {
            const int s = p / a.nq;
            const cx<T> f = Fr[(size_t)p * a.ld];
#pragma unroll
            for (int t = 0; t < WJB; ++t) {
                const int tt = j0 + t - s + 1;
                const bool ok = tt >= 0 && tt < KORD && j0 + t < a.nbz;
                const T w0 = a.wbz[(size_t)p * KORD + (ok ? tt : 0)];
                rfma(v[t], ok ? w0 : (T)0, f);
            }
        }
    }
    if (a.proj) {
        for (int k = a.ploff[i]; k < a.ploff[i + 1]; ++k) {
            const int q = a.plist[k];
            const int z0 = a.zwin[2 * q], z1 = a.zwin[2 * q + 1];
            if (z1 < j0 || z0 >= j0 + WJB) continue;
            cx<T> cf = mk<T>(0, 0);
            cfma(cf, a.Fp[(size_t)q * a.ld + g], a.proj[(size_t)b * a.np + q]);
            cf = cscale(cf, a.X[(size_t)q * a.nbx + i]);
#pragma unroll
            for (int t = 0; t < WJB; ++t) {
                const int j = j0 + t;
                if (j < z0 || j > z1) continue;
                rfma(v[t], a.Z[(size_t)q * a.nbz + j], cf);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < WJB; ++t) {
        if (t >= nj) continue;
        a.y[ob + (size_t)t * a.ld] = mk<TI>((TI)(kin[t].x + (double)v[t].x), (TI)(kin[t].y + (double)v[t].y));
        if (a.sy) a.sy[ob + (size_t)t * a.ld] = mk<TI>((TI)sc[t].x, (TI)sc[t].y);
    }
}

// launches the combine over band chunks of at most 65,535 (grid z limit); z rows per
// thread: 4 (MBKS_WIRE_COMBINE_ROWS=8 selects 8: 181 against 108 VGPRs, slower on the
// 19-line ribbon, 3.5 against 2.7 ms per 96 bands in FP64)
template <typename TI, typename T, int WJB>
mb_status launch_wire_combine_jb(WCombineArgs<TI, T> a, hipStream_t s) {
    const int64_t n = (int64_t)a.nbx * a.ld;
    const int njc = (a.nbz + WJB - 1) / WJB;
    const size_t vstride = (size_t)a.nbx * a.nbz * a.ld, fstride = (size_t)a.nbx * a.nzq * a.ld;
    const int total = a.nbands;
    for (int b0 = 0; b0 < total; b0 += 65535) {
        WCombineArgs<TI, T> c = a;
        c.nbands = std::min(65535, total - b0);
        c.c = a.c + b0 * vstride;
        c.y = a.y + b0 * vstride;
        if (a.sy) c.sy = a.sy + b0 * vstride;
        if (a.F) c.F = a.F + b0 * fstride;
        if (a.proj) c.proj = a.proj + (size_t)b0 * a.np;
        hipLaunchKernelGGL((k_wire_combine<TI, T, WJB>), dim3((unsigned)((n + 255) / 256), njc, c.nbands), dim3(256),
                           0, s, c);
        MB_HIP_TRY(hipGetLastError());
    }
    return MB_OK;
}

template <typename TI, typename T>
mb_status launch_wire_combine(const WCombineArgs<TI, T>& a, hipStream_t s) {
    const char* sel = getenv("MBKS_WIRE_COMBINE_ROWS");
    if (sel && std::string(sel) == "8") return launch_wire_combine_jb<TI, T, 8>(a, s);
    return launch_wire_combine_jb<TI, T, 4>(a, s);
}

// ---- banded substitutions -----------------------------------------------------------------
// Solve L L^T x = r along one direction: n rows at stride `st` (complex elements), band
// factor lf[row][d] = L[row][row - d] at stride lstride per row (per-line factors: the
// caller offsets lf); FP64 arithmetic.
template <typename TI>
__device__ void band_solve_strided(const cx<TI>* r, cx<TI>* x, size_t st, int n, const double* lf, size_t lrow,
                                   size_t ld_, double theta, const cx<TI>* sv) {
    auto L = [&](int row, int d) -> double { return lf[(size_t)row * lrow + (size_t)d * ld_]; };
    cx<double> h1 = mk<double>(0, 0), h2 = h1, h3 = h1;
    for (int i = 0; i < n; ++i) {
        const cx<TI> rv = r[(size_t)i * st];
        double ar = (double)rv.x, ai = (double)rv.y;
        if (sv) {
            const cx<TI> s = sv[(size_t)i * st];
            ar -= theta * (double)s.x;
            ai -= theta * (double)s.y;
        }
        const double l1 = i >= 1 ? L(i, 1) : 0.0, l2 = i >= 2 ? L(i, 2) : 0.0, l3 = i >= 3 ? L(i, 3) : 0.0;
        ar -= l1 * h1.x + l2 * h2.x + l3 * h3.x;
        ai -= l1 * h1.y + l2 * h2.y + l3 * h3.y;
        const double inv = 1.0 / L(i, 0);
        h3 = h2;
        h2 = h1;
        h1 = mk<double>(ar * inv, ai * inv);
        x[(size_t)i * st] = mk<TI>((TI)h1.x, (TI)h1.y);
    }
    // backward: L^T x = w, L^T[i][i+d] = L[i+d][i] = lf[i+d][d]
    h1 = mk<double>(0, 0);
    h2 = h1;
    h3 = h1;
    for (int i = n - 1; i >= 0; --i) {
        const cx<TI> wv = x[(size_t)i * st];
        double ar = (double)wv.x, ai = (double)wv.y;
        const double u1 = i + 1 < n ? L(i + 1, 1) : 0.0, u2 = i + 2 < n ? L(i + 2, 2) : 0.0,
                     u3 = i + 3 < n ? L(i + 3, 3) : 0.0;
        ar -= u1 * h1.x + u2 * h2.x + u3 * h3.x;
        ai -= u1 * h1.y + u2 * h2.y + u3 * h3.y;
        const double inv = 1.0 / L(i, 0);
        h3 = h2;
        h2 = h1;
        h1 = mk<double>(ar * inv, ai * inv);
        x[(size_t)i * st] = mk<TI>((TI)h1.x, (TI)h1.y);
    }
}

// x = S_x^{-1} r along x for every (band, j, G); then S_z^{-1} along z for every (band, i, G)
template <typename TI>
__global__ void k_wire_solve_x(const cx<TI>* r, cx<TI>* x, const double* lx, int nbands, int ld, int ng, int nbx,
                               int nbz) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (o >= (int64_t)nbz * ld) return;
    const int j = (int)(o / ld), g = (int)(o - (int64_t)j * ld);
    const size_t base = (size_t)b * nbx * nbz * ld + (size_t)j * ld + g;
    const size_t st = (size_t)nbz * ld;
    if (g >= ng) {
        for (int i = 0; i < nbx; ++i) x[base + i * st] = mk<TI>(0, 0);
        return;
    }
    band_solve_strided<TI>(r + base, x + base, st, nbx, lx, KORD, 1, 0.0, nullptr);
}

template <typename TI>
__global__ void k_wire_solve_z(cx<TI>* x, const double* lz, int nbands, int ld, int ng, int nbx, int nbz) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (o >= (int64_t)nbx * ld) return;
    const int i = (int)(o / ld), g = (int)(o - (int64_t)i * ld);
    if (g >= ng) return;
    const size_t base = ((size_t)b * nbx + i) * nbz * ld + g;
    band_solve_strided<TI>(x + base, x + base, (size_t)ld, nbz, lz, KORD, 1, 0.0, nullptr);
}

// ---- preconditioner -------------------------------------------------------------------------
// factors per (z eigenvector jp, G): banded Cholesky along x of
// kin (1/2 D_x + (lambda_jp / 2 + |k+G|^2 / 2) S_x) + shift S_x; pf[((jp nbx + i) kappa + d) ld + g]
__global__ void k_wire_prec_factor(double* pf, const double* sx, const double* dx, const double* lamz,
                                   const double* kg2, double kin, double shift, int ng, int ld, int nbx, int nbz,
                                   int* fail) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= (int64_t)nbz * ng) return;
    const int jp = (int)(o / ng), g = (int)(o - (int64_t)jp * ng);
    const double sh = kin * 0.5 * (lamz[jp] + kg2[g]) + shift;
    auto M = [&](int i, int i2) -> double { return kin * 0.5 * band_at(dx, i, i2) + sh * band_at(sx, i, i2); };
    double* base = pf + (size_t)jp * nbx * KORD * ld + g;
    auto Lr = [&](int i, int j) -> double& { return base[((size_t)i * KORD + (i - j)) * ld]; };
    for (int i = 0; i < nbx; ++i) {
        const int j0 = max(0, i - (KORD - 1));
        for (int j = j0; j <= i; ++j) {
            double sum = M(i, j);
            for (int k = max(j0, j - (KORD - 1)); k < j; ++k) sum -= Lr(i, k) * Lr(j, k);
            if (j == i) {
                if (!(sum > 0)) {
                    atomicExch(fail, 1);
                    sum = 1.0;
                }
                Lr(i, i) = sqrt(sum);
            } else {
                Lr(i, j) = sum / Lr(j, j);
            }
        }
        for (int d = i + 1; d < KORD; ++d) base[((size_t)i * KORD + d) * ld] = 0.0;
    }
}

// tmp[v][i][jp][G] = sum_j Uz[j][jp] (h - theta s)[sel v][i][j][G]; one workgroup per (i, v)
__global__ __launch_bounds__(WNT) void k_wire_prec_fwd(const cx<double>* h, const cx<double>* sv,
                                                       const double* theta, const int32_t* sel, cx<double>* tmp,
                                                       const double* Uz, int ld, int ng, int nbx, int nbz) {
    extern __shared__ unsigned char smem_raw[];
    cx<double>* r = reinterpret_cast<cx<double>*>(smem_raw);  // [nbz][ng]
    const int i = blockIdx.x, v = blockIdx.y;
    const int src = sel ? sel[v] : v;
    const double th = theta ? theta[v] : 0.0;
    const size_t in = ((size_t)src * nbx + i) * nbz * ld;
    for (int o = threadIdx.x; o < nbz * ng; o += WNT) {
        const int j = o / ng, g = o - j * ng;
        cx<double> a = h[in + (size_t)j * ld + g];
        if (sv) {
            const cx<double> s = sv[in + (size_t)j * ld + g];
            a.x -= th * s.x;
            a.y -= th * s.y;
        }
        r[o] = a;
    }
    __syncthreads();
    const size_t outb = ((size_t)v * nbx + i) * nbz * ld;
    for (int o = threadIdx.x; o < nbz * ng; o += WNT) {
        const int jp = o / ng, g = o - jp * ng;
        cx<double> acc = mk<double>(0, 0);
        for (int j = 0; j < nbz; ++j) rfma(acc, Uz[(size_t)j * nbz + jp], r[j * ng + g]);
        tmp[outb + (size_t)jp * ld + g] = acc;
    }
}

// banded x solve of the preconditioner, in place on tmp, one thread per (v, jp, G)
__global__ void k_wire_prec_xsolve(cx<double>* tmp, const double* pf, int ld, int ng, int nbx, int nbz) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y;
    if (o >= (int64_t)nbz * ng) return;
    const int jp = (int)(o / ng), g = (int)(o - (int64_t)jp * ng);
    cx<double>* base = tmp + (size_t)v * nbx * nbz * ld + (size_t)jp * ld + g;
    band_solve_strided<double>(base, base, (size_t)nbz * ld, nbx, pf + (size_t)jp * nbx * KORD * ld + g,
                               (size_t)KORD * ld, (size_t)ld, 0.0, nullptr);
}

// x[v][i][j][G] = sum_jp Uz[j][jp] tmp[v][i][jp][G]; padding G >= ng set to zero
__global__ __launch_bounds__(WNT) void k_wire_prec_bwd(const cx<double>* tmp, cx<double>* x, const double* Uz,
                                                       int ld, int ng, int nbx, int nbz) {
    extern __shared__ unsigned char smem_raw[];
    cx<double>* a = reinterpret_cast<cx<double>*>(smem_raw);
    const int i = blockIdx.x, v = blockIdx.y;
    const size_t base = ((size_t)v * nbx + i) * nbz * ld;
    for (int o = threadIdx.x; o < nbz * ng; o += WNT) {
        const int jp = o / ng, g = o - jp * ng;
        a[o] = tmp[base + (size_t)jp * ld + g];
    }
    __syncthreads();
    for (int o = threadIdx.x; o < nbz * ld; o += WNT) {
        const int j = o / ld, g = o - j * ld;
        cx<double> acc = mk<double>(0, 0);
        if (g < ng)
            for (int jp = 0; jp < nbz; ++jp) rfma(acc, Uz[(size_t)j * nbz + jp], a[jp * ng + g]);
        x[base + (size_t)j * ld + g] = acc;
    }
}

template <typename TI, typename T>
mb_status wire_apply_t(Problem* p, int ik, const void* c, void* y, void* sy, int nbands, int ld, hipStream_t s,
                       bool lowT) {
    WireTables& w = *p->wire;
    KPoint& kp = p->kp[ik];
    const bool dbl = sizeof(T) == 8;
    const int nbx = w.x.nb, nbz = w.z.nb;
    const size_t fbytes = (size_t)nbands * nbx * w.z.nzq * ld * sizeof(cx<T>);
    MB_TRY(ensure_hws(kp, kp.ws_part, fbytes));
    cx<T>* proj = nullptr;
    if (p->np > 0) {
        MB_TRY(ensure_hws(kp, kp.ws_proj, (size_t)nbands * p->np * sizeof(cx<T>)));
        proj = (cx<T>*)kp.ws_proj.ptr;
        StageScope ts_(MB_STAGE_NL_PROJECT, s, nbands);
        hipLaunchKernelGGL((k_wire_nlproj<TI, T>), dim3(p->np, nbands), dim3(WNT), 0, s, (const cx<TI>*)c, proj,
                           (const cx<T>*)(dbl ? kp.d_F64 : kp.d_F32), (const T*)(dbl ? (void*)w.d_X : (void*)w.d_Xf),
                           (const T*)(dbl ? (void*)w.d_Z : (void*)w.d_Zf), (const T*)(dbl ? (void*)p->d_E : (void*)p->d_Ef),
                           w.d_xwin, w.d_zwin, nbands, ld, kp.ng, nbx, nbz, p->np);
        MB_HIP_TRY(hipGetLastError());
    }
    {
        WLocalArgs<TI, T> a;
        a.c = (const cx<TI>*)c;
        a.F = (cx<T>*)kp.ws_part.ptr;
        a.bx = (const T*)(dbl ? (void*)w.d_bx : (void*)w.d_bxf);
        a.wbx = (const T*)(dbl ? (void*)w.d_wbx : (void*)w.d_wbxf);
        a.bz = (const T*)(dbl ? (void*)w.d_bz : (void*)w.d_bzf);
        a.V = (const T*)(dbl ? (void*)w.d_V : (void*)w.d_Vf);
        a.tw = (const cx<T>*)(dbl ? w.d_tw : w.d_twf);
        a.gtab = kp.d_gtab;
        a.nbands = nbands;
        a.ld = ld;
        a.ng = kp.ng;
        a.nbx = nbx;
        a.nbz = nbz;
        a.nintx = w.x.nint;
        a.nq = w.x.nq;
        a.nxq = w.x.nzq;
        a.nzq = w.z.nzq;
        StageScope ts_(lowT ? MB_STAGE_LOCAL32 : MB_STAGE_LOCAL, s, nbands);
        MB_TRY((wire_local_dispatch<TI, T>(a, w.ny, s)));
    }
    WCombineArgs<TI, T> a;
    a.c = (const cx<TI>*)c;
    a.F = (const cx<T>*)kp.ws_part.ptr;
    a.proj = proj;
    a.y = (cx<TI>*)y;
    a.sy = (cx<TI>*)sy;
    a.wbz = (const T*)(dbl ? (void*)w.d_wbz : (void*)w.d_wbzf);
    a.sx = w.d_sx;
    a.dx = w.d_dx;
    a.sz = w.d_sz;
    a.dz = w.d_dz;
    a.kg2 = kp.d_kg2;
    a.Fp = (const cx<T>*)(dbl ? kp.d_F64 : kp.d_F32);
    a.X = (const T*)(dbl ? (void*)w.d_X : (void*)w.d_Xf);
    a.Z = (const T*)(dbl ? (void*)w.d_Z : (void*)w.d_Zf);
    a.zwin = w.d_zwin;
    a.ploff = w.d_ploff;
    a.plist = w.d_plist;
    a.nbands = nbands;
    a.ld = ld;
    a.ng = kp.ng;
    a.nbx = nbx;
    a.nbz = nbz;
    a.nintz = w.z.nint;
    a.nq = w.z.nq;
    a.nzq = w.z.nzq;
    a.np = p->np;
    a.s_only = 0;
    StageScope ts_(MB_STAGE_COMBINE, s, nbands);
    return launch_wire_combine<TI, T>(a, s);
}

template <typename TI>
mb_status wire_spsi_t(Problem* p, int ik, const void* c, void* y, int nbands, int ld, hipStream_t s) {
    WireTables& w = *p->wire;
    KPoint& kp = p->kp[ik];
    WCombineArgs<TI, TI> a{};
    a.c = (const cx<TI>*)c;
    a.y = (cx<TI>*)y;
    a.sx = w.d_sx;
    a.dx = w.d_dx;
    a.sz = w.d_sz;
    a.dz = w.d_dz;
    a.kg2 = kp.d_kg2;
    a.nbands = nbands;
    a.ld = ld;
    a.ng = kp.ng;
    a.nbx = w.x.nb;
    a.nbz = w.z.nb;
    a.nintz = w.z.nint;
    a.nq = w.z.nq;
    a.nzq = w.z.nzq;
    a.np = p->np;
    a.s_only = 1;
    StageScope ts_(MB_STAGE_SPSI, s, nbands);
    return launch_wire_combine<TI, TI>(a, s);
}

template <typename TI>
mb_status wire_ssolve_t(Problem* p, int ik, const void* r, void* x, int nbands, int ld, hipStream_t s) {
    WireTables& w = *p->wire;
    KPoint& kp = p->kp[ik];
    StageScope ts_(MB_STAGE_SSOLVE, s, nbands);
    const int64_t nx = (int64_t)w.z.nb * ld, nz = (int64_t)w.x.nb * ld;
    hipLaunchKernelGGL((k_wire_solve_x<TI>), dim3((unsigned)((nx + 127) / 128), nbands), dim3(128), 0, s,
                       (const cx<TI>*)r, (cx<TI>*)x, w.d_lx, nbands, ld, kp.ng, w.x.nb, w.z.nb);
    MB_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL((k_wire_solve_z<TI>), dim3((unsigned)((nz + 127) / 128), nbands), dim3(128), 0, s,
                       (cx<TI>*)x, w.d_lz, nbands, ld, kp.ng, w.x.nb, w.z.nb);
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

}  // namespace

mb_status upload_wire(Problem* p) {
    WireTables& w = *p->wire;
    MB_TRY(put(&w.d_bx, w.x.bval));
    MB_TRY(putf(&w.d_bxf, w.x.bval));
    MB_TRY(put(&w.d_wbx, w.x.wbval));
    MB_TRY(putf(&w.d_wbxf, w.x.wbval));
    MB_TRY(put(&w.d_bz, w.z.bval));
    MB_TRY(putf(&w.d_bzf, w.z.bval));
    MB_TRY(put(&w.d_wbz, w.z.wbval));
    MB_TRY(putf(&w.d_wbzf, w.z.wbval));
    MB_TRY(put(&w.d_sx, w.x.sband));
    MB_TRY(put(&w.d_dx, w.x.dband));
    MB_TRY(put(&w.d_lx, w.x.lband));
    MB_TRY(put(&w.d_sz, w.z.sband));
    MB_TRY(put(&w.d_dz, w.z.dband));
    MB_TRY(put(&w.d_lz, w.z.lband));
    MB_TRY(put(&w.d_Uz, w.Uz));
    MB_TRY(put(&w.d_lamz, w.lamz));
    if (p->np > 0) {
        MB_TRY(put(&w.d_X, w.Xp));
        MB_TRY(putf(&w.d_Xf, w.Xp));
        MB_TRY(put(&w.d_Z, w.Zp));
        MB_TRY(putf(&w.d_Zf, w.Zp));
        MB_TRY(put(&w.d_xwin, w.xwin));
        MB_TRY(put(&w.d_zwin, w.zwin));
        MB_TRY(put(&p->d_E, p->Ep));
        MB_TRY(putf(&p->d_Ef, p->Ep));
    }
    MB_TRY(put(&w.d_ploff, w.ploff));
    if (!w.plist.empty()) MB_TRY(put(&w.d_plist, w.plist));
    {
        std::vector<cx<double>> t(w.ny);
        std::vector<cx<float>> tf(w.ny);
        for (int k = 0; k < w.ny; ++k) {
            const double a = 2.0 * 3.14159265358979323846 * k / w.ny;
            t[k] = mk<double>(std::cos(a), std::sin(a));
            tf[k] = mk<float>((float)t[k].x, (float)t[k].y);
        }
        MB_TRY(put((cx<double>**)&w.d_tw, t));
        MB_TRY(put((cx<float>**)&w.d_twf, tf));
    }
    for (auto& kp : p->kp) {
        MB_TRY(put(&kp.d_kg2, kp.kg2));
        MB_TRY(putf(&kp.d_kg2f, kp.kg2));
        MB_TRY(put(&kp.d_gtab, kp.gtab));
        if (p->np > 0) {
            std::vector<cx<double>> F(kp.F.size());
            std::vector<cx<float>> Ff(kp.F.size());
            for (size_t e = 0; e < kp.F.size(); ++e) {
                F[e] = mk<double>(kp.F[e].real(), kp.F[e].imag());
                Ff[e] = mk<float>((float)kp.F[e].real(), (float)kp.F[e].imag());
            }
            MB_TRY(put((cx<double>**)&kp.d_F64, F));
            MB_TRY(put((cx<float>**)&kp.d_F32, Ff));
        }
    }
    // the potential on (z_p, x_q, y_n)
    std::vector<WTerm> terms;
    for (const auto& at : p->atoms) {
        const mb_species& sp = p->species[at.species];
        for (int t = 0; t < sp.ngauss; ++t) {
            WTerm tm;
            tm.A = sp.gauss_A[t];
            tm.w = sp.gauss_w[t];
            tm.X = at.pos[0];
            tm.Y = at.pos[1];
            tm.Z = at.pos[2];
            tm.nimg = (int)std::ceil(std::sqrt(45.0) * tm.w / w.period) + 1;
            terms.push_back(tm);
        }
    }
    const size_t nv = (size_t)w.z.nzq * w.x.nzq * w.ny;
    if (hipMalloc(&w.d_V, nv * sizeof(double)) != hipSuccess) return set_error(MB_ERR_OOM, "potential grid");
    if (hipMalloc(&w.d_Vf, nv * sizeof(float)) != hipSuccess) return set_error(MB_ERR_OOM, "potential grid");
    WTerm* d_terms = nullptr;
    double *d_xq = nullptr, *d_zq = nullptr;
    MB_TRY(put(&d_xq, w.x.zq));
    MB_TRY(put(&d_zq, w.z.zq));
    if (!terms.empty()) MB_TRY(put(&d_terms, terms));
    hipLaunchKernelGGL(k_wire_vgrid, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, 0, w.d_V, w.d_Vf, d_xq, d_zq,
                       d_terms, (int)terms.size(), w.x.nzq, w.z.nzq, w.ny, w.period);
    MB_HIP_TRY(hipGetLastError());
    MB_HIP_TRY(hipDeviceSynchronize());
    (void)hipFree(d_xq);
    (void)hipFree(d_zq);
    if (d_terms) (void)hipFree(d_terms);
    return MB_OK;
}

void free_wire(Problem* p) {
    if (!p->wire) return;
    WireTables& w = *p->wire;
    if (p->device >= 0) {
        void* ptrs[] = {w.d_bx, w.d_wbx, w.d_bz, w.d_wbz, w.d_bxf, w.d_wbxf, w.d_bzf, w.d_wbzf, w.d_sx, w.d_dx,
                        w.d_lx, w.d_sz, w.d_dz, w.d_lz, w.d_X, w.d_Z, w.d_Xf, w.d_Zf, w.d_xwin, w.d_zwin,
                        w.d_ploff, w.d_plist, w.d_Uz, w.d_lamz, w.d_V, w.d_Vf, w.d_tw, w.d_twf};
        for (void* q : ptrs)
            if (q) (void)hipFree(q);
    }
    delete p->wire;
    p->wire = nullptr;
}

mb_status wire_apply_h(Problem* p, int ik, const void* c, void* y, void* sy, int nbands, int ld, int lp,
                       hipStream_t s) {
    if (nbands == 0) return MB_OK;
    if (lp == 0) return wire_apply_t<double, double>(p, ik, c, y, sy, nbands, ld, s, false);
    if (lp == 1) return wire_apply_t<float, float>(p, ik, c, y, sy, nbands, ld, s, true);
    return wire_apply_t<double, float>(p, ik, c, y, sy, nbands, ld, s, true);
}

mb_status wire_spsi(Problem* p, int ik, const void* c, void* y, int nbands, int ld, int prec, hipStream_t s) {
    if (nbands == 0) return MB_OK;
    return prec == 0 ? wire_spsi_t<double>(p, ik, c, y, nbands, ld, s) : wire_spsi_t<float>(p, ik, c, y, nbands, ld, s);
}

mb_status wire_ssolve(Problem* p, int ik, const void* r, void* x, int nbands, int ld, int prec, hipStream_t s) {
    if (nbands == 0) return MB_OK;
    return prec == 0 ? wire_ssolve_t<double>(p, ik, r, x, nbands, ld, s)
                     : wire_ssolve_t<float>(p, ik, r, x, nbands, ld, s);
}

mb_status wire_prec_factor(Problem* p, int ik, double sigma, hipStream_t s) {
    KPoint& kp = p->kp[ik];
    WireTables& w = *p->wire;
    if (kp.d_pfac && kp.pfac_sigma == sigma) return MB_OK;
    if (!kp.d_pfac)
        MB_HIP_TRY(hipMalloc(&kp.d_pfac, (size_t)w.z.nb * w.x.nb * KORD * kp.ld * sizeof(double)));
    int* d_fail = nullptr;
    MB_HIP_TRY(hipMalloc(&d_fail, sizeof(int)));
    MB_HIP_TRY(hipMemsetAsync(d_fail, 0, sizeof(int), s));
    // sigma > 0: (T + sigma S)^{-1}; sigma <= 0: S^{-1}
    const double kin = sigma > 0 ? 1.0 : 0.0, shift = sigma > 0 ? sigma : 1.0;
    const int64_t n = (int64_t)w.z.nb * kp.ng;
    hipLaunchKernelGGL(k_wire_prec_factor, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, kp.d_pfac, w.d_sx,
                       w.d_dx, w.d_lamz, kp.d_kg2, kin, shift, kp.ng, kp.ld, w.x.nb, w.z.nb, d_fail);
    MB_HIP_TRY(hipGetLastError());
    int fail = 0;
    MB_HIP_TRY(hipMemcpyAsync(&fail, d_fail, sizeof(int), hipMemcpyDeviceToHost, s));
    MB_HIP_TRY(hipStreamSynchronize(s));
    MB_HIP_TRY(hipFree(d_fail));
    if (fail) return set_error(MB_ERR_NOT_SPD, "preconditioner block not positive definite");
    kp.pfac_sigma = sigma;
    return MB_OK;
}

mb_status wire_prec_apply(Problem* p, int ik, const void* h, const void* sv, const double* theta, const int32_t* sel,
                          void* x, int nvec, int ld, hipStream_t s) {
    KPoint& kp = p->kp[ik];
    WireTables& w = *p->wire;
    if (!kp.d_pfac || ld != kp.ld) return set_error(MB_ERR_INVALID_ARG, "preconditioner not built for this ld");
    if (nvec == 0) return MB_OK;
    const int nbx = w.x.nb, nbz = w.z.nb;
    const size_t lds = (size_t)nbz * kp.ng * sizeof(cx<double>);
    if (lds > 160 * 1024) return set_error(MB_ERR_INVALID_ARG, "1D-periodic preconditioner: z rows x G too large for LDS");
    MB_TRY(ensure_ws(kp.ws_aux, (size_t)nvec * nbx * nbz * ld * sizeof(cx<double>)));
    cx<double>* tmp = (cx<double>*)kp.ws_aux.ptr;
    StageScope ts_(MB_STAGE_PRECOND, s, nvec);
    if (lds > 64 * 1024) {
        MB_HIP_TRY(hipFuncSetAttribute((const void*)k_wire_prec_fwd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        MB_HIP_TRY(hipFuncSetAttribute((const void*)k_wire_prec_bwd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    }
    hipLaunchKernelGGL(k_wire_prec_fwd, dim3(nbx, nvec), dim3(WNT), lds, s, (const cx<double>*)h,
                       (const cx<double>*)sv, theta, sel, tmp, w.d_Uz, ld, kp.ng, nbx, nbz);
    MB_HIP_TRY(hipGetLastError());
    const int64_t n = (int64_t)nbz * kp.ng;
    hipLaunchKernelGGL(k_wire_prec_xsolve, dim3((unsigned)((n + 63) / 64), nvec), dim3(64), 0, s, tmp, kp.d_pfac, ld,
                       kp.ng, nbx, nbz);
    MB_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_wire_prec_bwd, dim3(nbx, nvec), dim3(WNT), lds, s, (const cx<double>*)tmp, (cx<double>*)x,
                       w.d_Uz, ld, kp.ng, nbx, nbz);
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

}  // namespace mb
