// Local-potential part of H c, one Gauss plane at a time, for in-plane grids whose FFT
// lines are split over a few lanes (the 128 x 64 grid of the large surface slab, and the
// 36 x 36 grid of the graphene-like slab):
//   evaluate psi(G, z_q) = sum_t B_{s-1+t}(z_q) c(G, s-1+t), scatter on the sphere rows,
//   inverse 2D FFT, multiply by V(rho, z_q), forward 2D FFT, gather, and write
//   u_q(G) = (V psi_q)(G) / (N1 N2) for every Gauss plane q (local-potential matrix
//   elements of Sec. II.B.1, taken on the grid); the combine pass projects the planes
//   onto the spline rows, sum_q w_q B_i(z_q) u_q(G).
// Every line of N = Q L points is held by Q neighbouring lanes, lane l owning the
// points l + Q m (m < L).  Inverse transform: an L-point register FFT per lane, the
// twiddle w_N^{l k}, then a radix-2 decimation-in-frequency network across the Q lanes
// (lane exchanges), which leaves lane l holding the outputs k + L bitrev(l).  Forward
// transform: the mirrored decimation-in-time network across the lanes, the conjugate
// twiddle and the L-point register FFT, which returns the points l + Q m to lane l.  A
// plane takes two passes through LDS: rows (only the rows that hold sphere points) and
// columns; the potential multiply sits inside the column pass.  No thread keeps
// accumulators across planes, so no registers spill at any plane count.
#include <algorithm>
#include <cstring>
#include <vector>

#include "cplx.h"
#include "fft_line.h"
#include "lane_fft.h"
#include "mbks_internal.h"

namespace mb {

namespace {

constexpr int KORD = 4;
constexpr int PLANE_BG = 8;  // bands per group of the work order
// consecutive knot intervals per workgroup: 1.  With 4, each workgroup re-reads fewer
// rows itself, but the rows resident on an XCD (8 bands x 8 chunks x 4 intervals) no
// longer fit its L2 and the HBM fetch per 320-band launch of the surface slab rose from
// 11.3 GB to 46.7 GB (measured)
constexpr int PLANE_NI = 1;
using fftl::line_fft;

template <typename TI, typename T>
struct PlaneArgs {
    const cx<TI>* c;       // [b][i][ld]
    cx<T>* u;              // [b][q][ld]: (V psi_q)(G) / (N1 N2)
    const T* bval;         // [q][kappa]
    const T* Vt;           // [q][j2][j1]: the potential with the in-plane axes swapped
    const int32_t* gtab;   // [nrows][N2]: G index at (sphere row, column), -1 outside the sphere
    const int32_t* rows;   // [nrows]: grid row j1 of each sphere row
    const cx<T>* tw1;      // [N1]: exp(+2 pi i k / N1)
    const cx<T>* tw2;      // [N2]
    int nbands, ld, nint, nq, nb, nrows, nzq;
    int nreal;             // real-wavefunction pairing: bands (nbands counts the pairs)
    T inv_n;
};

// LDS row pitch and column position: columns are stored in blocks of L2 with PADB
// elements after each block, so the Q2 lanes of a row write their blocks to different banks
template <int N2, int Q2, int PADB>
constexpr int plane_pitch() { return N2 + Q2 * PADB + 1; }

template <int N2, int Q2, int PADB>
__device__ __forceinline__ int colpos(int j2) {
    return j2 + (j2 / (N2 / Q2)) * PADB;
}

template <typename T, int N1, int N2>
constexpr size_t plane_hdr() {
    return ((sizeof(cx<T>) * (N1 + N2) + sizeof(uint32_t) * ((N1 + 31) / 32) + 255) / 256) * 256;
}

template <typename T, int N1, int N2, int Q2, int PADB>
constexpr size_t plane_lds() {
    return plane_hdr<T, N1, N2>() + sizeof(cx<T>) * (size_t)N1 * plane_pitch<N2, Q2, PADB>();
}

// One workgroup per (band, chunk of PLANE_NI knot intervals): their Gauss planes one
// after another.
// GAM: real wavefunctions at the Gamma point (c(-G) = conj c(G), so psi(rho, z) is real):
// one complex transform serves two bands.  Work band b is the pair (2b, 2b + 1); the
// row pass evaluates psi_2b + i psi_2b+1, the real potential keeps the two parts apart
// in real space, and after the forward transform u = A + i B with A(-G) = conj A(G),
// B(-G) = conj B(G), so A(G) = (u(G) + conj u(-G)) / 2 and B(G) = (u(G) - conj u(-G)) / 2i.
// The forward row pass leaves the plane in LDS, and a gather pass reads G and -G.
template <typename TI, typename T, int N1, int N2, int Q1, int Q2, int NT, int PADB, bool GAM>
__global__ __launch_bounds__(NT) void k_local_plane(PlaneArgs<TI, T> a) {
    constexpr int L1 = N1 / Q1, L2 = N2 / Q2;
    constexpr int P = plane_pitch<N2, Q2, PADB>();
    extern __shared__ unsigned char smem_raw[];
    cx<T>* tw1 = reinterpret_cast<cx<T>*>(smem_raw);
    cx<T>* tw2 = tw1 + N1;
    uint32_t* rmask = reinterpret_cast<uint32_t*>(tw2 + N2);
    cx<T>* grid = reinterpret_cast<cx<T>*>(smem_raw + plane_hdr<T, N1, N2>());

    // Work order: a workgroup takes PLANE_NI consecutive knot intervals of one band.
    // Groups of PLANE_BG bands walk the interval chunks together, the bands of a group
    // side by side; consecutive logical workgroups share an XCD, so the workgroups
    // resident on one XCD cover a few bands x neighbouring intervals: a band's
    // coefficient rows (used by the kappa intervals around them) and an interval's
    // potential planes (used by every band of the group) stay in its L2.
    const unsigned L = xcd_logical(blockIdx.x, gridDim.x);
    const int nch = (a.nint + PLANE_NI - 1) / PLANE_NI;
    const unsigned full = (unsigned)(a.nbands / PLANE_BG) * PLANE_BG;
    const unsigned span = (unsigned)PLANE_BG * (unsigned)nch;
    int b, ch;
    if (L < full * (unsigned)nch) {
        const unsigned r = L % span;
        b = (int)((L / span) * PLANE_BG + r % PLANE_BG);
        ch = (int)(r / PLANE_BG);
    } else {
        const unsigned rb = (unsigned)a.nbands - full, r = L - full * (unsigned)nch;
        b = (int)(full + r % rb);
        ch = (int)(r / rb);
    }
    if (ch >= nch || b >= a.nbands) return;
    const int s_begin = ch * PLANE_NI, s_end = min(s_begin + PLANE_NI, a.nint);
    const int tid = threadIdx.x;
    for (int e = tid; e < N1; e += NT) tw1[e] = a.tw1[e];
    for (int e = tid; e < N2; e += NT) tw2[e] = a.tw2[e];
    for (int e = tid; e < (N1 + 31) / 32; e += NT) rmask[e] = 0u;
    __syncthreads();
    for (int e = tid; e < a.nrows; e += NT) {
        const int j1 = a.rows[e];
        atomicOr(&rmask[j1 >> 5], 1u << (j1 & 31));
    }
    __syncthreads();

    const int b0 = GAM ? 2 * b : b;
    const bool hasb = GAM && b0 + 1 < a.nreal;  // second band of the pair
    const cx<TI>* cb = a.c + (size_t)b0 * a.nb * a.ld;
    const cx<TI>* cb2 = hasb ? cb + (size_t)a.nb * a.ld : cb;  // weight 0 if absent
    cx<T>* ub = a.u + (size_t)b0 * a.nzq * a.ld;
    // row tasks in whole 16-lane rows (a line's lanes are active or idle together)
    const int nrt = (a.nrows * Q2 + 15) / 16 * 16;

    for (int q = s_begin * a.nq; q < s_end * a.nq; ++q) {
        const int s = q / a.nq;
        T bv[KORD];
#pragma unroll
        for (int t = 0; t < KORD; ++t) bv[t] = a.bval[(size_t)q * KORD + t];

        // rows: evaluate on the sphere row, inverse transform along j2
        for (int task = tid; task < nrt; task += NT) {
            const int rc = (task >> 4) * (16 / Q2) + LaneMap<Q2>::line(task & 15);
            const int l = LaneMap<Q2>::lane(task & 15);
            if (rc >= a.nrows) continue;
            const int j1 = a.rows[rc];
            const int32_t* gr = a.gtab + (size_t)rc * N2;
            cx<T> x[L2];
            int gi[L2];
#pragma unroll
            for (int m = 0; m < L2; ++m) {
                gi[m] = gr[l + Q2 * m];
                x[m] = mk<T>(0, 0);
            }
            // one spline row at a time keeps L2 loads in flight, not kappa L2
#pragma unroll 1
            for (int t = 0; t < KORD; ++t) {
                const int row = s - 1 + t;
                if (row < 0 || row >= a.nb) continue;
                const cx<TI>* cr = cb + (size_t)row * a.ld;
#pragma unroll
                for (int m = 0; m < L2; ++m) {
                    // off the sphere: load G = 0 and weigh it by zero (no branch)
                    const cx<TI> v = cr[gi[m] >= 0 ? gi[m] : 0];
                    const T w = gi[m] >= 0 ? bv[t] : (T)0;
                    x[m].x = fma(w, (T)v.x, x[m].x);
                    x[m].y = fma(w, (T)v.y, x[m].y);
                    if constexpr (GAM) {  // + i c of the pair's second band
                        const cx<TI> v2 = cb2[(size_t)row * a.ld + (gi[m] >= 0 ? gi[m] : 0)];
                        const T w2 = hasb ? w : (T)0;
                        x[m].x = fma(-w2, (T)v2.y, x[m].x);
                        x[m].y = fma(w2, (T)v2.x, x[m].y);
                    }
                }
            }
            line_fft<T, L2, +1>(x);
#pragma unroll
            for (int k = 1; k < L2; ++k) x[k] = cmul(x[k], tw_at<T, +1>(tw2, l * k));
            // the last stage's sign (-1 on lanes with bit 0 set) stays on the values: it
            // marks the columns j2 >= N2 / 2, whose pass takes it into the potential
            dif_lanes<T, L2, Q2, N2, +1, true>(x, l, tw2);
            cx<T>* dst = grid + (size_t)j1 * P + colpos<N2, Q2, PADB>(L2 * bitrev_lane<Q2>(l));
#pragma unroll
            for (int k = 0; k < L2; ++k) dst[k] = x[k];
        }
        __syncthreads();

        // columns: inverse transform along j1, potential multiply, forward transform
        for (int task = tid; task < N2 * Q1; task += NT) {
            const int j2 = (task >> 4) * (16 / Q1) + LaneMap<Q1>::line(task & 15);
            const int l = LaneMap<Q1>::lane(task & 15);
            const int cp = colpos<N2, Q2, PADB>(j2);
            uint32_t live = 0u;
#pragma unroll
            for (int m = 0; m < L1; ++m) {
                const int j1 = l + Q1 * m;
                if ((rmask[j1 >> 5] >> (j1 & 31)) & 1u) live |= 1u << m;
            }
            // rows without sphere points hold stale data: read them and select zero
            cx<T> x[L1];
#pragma unroll
            for (int m = 0; m < L1; ++m) {
                const cx<T> v = grid[(size_t)(l + Q1 * m) * P + cp];
                x[m] = ((live >> m) & 1u) ? v : mk<T>(0, 0);
            }
            line_fft<T, L1, +1>(x);
#pragma unroll
            for (int k = 1; k < L1; ++k) x[k] = cmul(x[k], tw_at<T, +1>(tw1, l * k));
            // signs left on the values by folded last stages (+-1, products exact): the
            // row pass's (columns j2 >= N2 / 2) and this network's, both taken by V
            const T sgc = (lane_fold<T, 1, Q2>() && j2 >= N2 / 2) ? (T)-1 : (T)1;
            const T sv = sgc * dif_lanes<T, L1, Q1, N1, +1, true>(x, l, tw1);
            const T* vc = a.Vt + ((size_t)q * N2 + j2) * N1 + L1 * bitrev_lane<Q1>(l);
#pragma unroll
            for (int k = 0; k < L1; ++k) {
                const T v = sv * vc[k];
                x[k] = mk<T>(x[k].x * v, x[k].y * v);
            }
            // the forward network's last sign (lane bit 3, i.e. the rows j1 with bit 3 of
            // j1 mod Q1 set) goes on to the row pass, which takes it into its output scale
            dit_lanes<T, L1, Q1, N1, -1, true>(x, l, tw1);
#pragma unroll
            for (int k = 1; k < L1; ++k) x[k] = cmul(x[k], tw_at<T, -1>(tw1, l * k));
            line_fft<T, L1, -1>(x);
#pragma unroll
            for (int m = 0; m < L1; ++m) grid[(size_t)(l + Q1 * m) * P + cp] = x[m];
        }
        __syncthreads();

        // rows: forward transform along j2, gather the sphere points.  Each task reads
        // back exactly the LDS elements it wrote in the row pass above, so the next
        // plane's row pass needs no barrier before it.
        for (int task = tid; task < nrt; task += NT) {
            const int rc = (task >> 4) * (16 / Q2) + LaneMap<Q2>::line(task & 15);
            const int l = LaneMap<Q2>::lane(task & 15);
            if (rc >= a.nrows) continue;
            const int j1 = a.rows[rc];
            const int32_t* gr = a.gtab + (size_t)rc * N2;
            const cx<T>* src = grid + (size_t)j1 * P + colpos<N2, Q2, PADB>(L2 * bitrev_lane<Q2>(l));
            cx<T> x[L2];
#pragma unroll
            for (int k = 0; k < L2; ++k) x[k] = src[k];
            const T sr = dit_lanes<T, L2, Q2, N2, -1, true>(x, l, tw2);
#pragma unroll
            for (int k = 1; k < L2; ++k) x[k] = cmul(x[k], tw_at<T, -1>(tw2, l * k));
            line_fft<T, L2, -1>(x);
            // this network's last sign and the column pass's sign of row j1
            const T sj = (lane_fold<T, Q1 / 2, Q1>() && ((j1 % Q1) & (Q1 >> 1))) ? (T)-1 : (T)1;
            const T sc = a.inv_n * (sr * sj) * (GAM ? (T)0.5 : (T)1);
            if constexpr (GAM) {
                // the transformed row back to LDS in natural column order (this lane read
                // its own block above; the lanes of a row share one wavefront)
                cx<T>* dr = grid + (size_t)j1 * P;
#pragma unroll
                for (int m = 0; m < L2; ++m)
                    dr[colpos<N2, Q2, PADB>(l + Q2 * m)] = mk<T>(x[m].x * sc, x[m].y * sc);
            } else {
                cx<T>* uq = ub + (size_t)q * a.ld;
#pragma unroll
                for (int m = 0; m < L2; ++m) {
                    const int g = gr[l + Q2 * m];
                    if (g >= 0) uq[g] = mk<T>(x[m].x * sc, x[m].y * sc);
                }
            }
        }
        if constexpr (GAM) {
            // gather: the sphere is symmetric at Gamma, so -G sits on a sphere row too
            __syncthreads();
            cx<T>* uq = ub + (size_t)q * a.ld;
            cx<T>* uq2 = uq + (size_t)a.nzq * a.ld;
            for (int e = tid; e < a.nrows * N2; e += NT) {
                const int rc = e / N2, j2 = e - rc * N2;
                const int g = a.gtab[e];
                if (g < 0) continue;
                const int j1 = a.rows[rc];
                const int n1 = j1 == 0 ? 0 : N1 - j1, n2 = j2 == 0 ? 0 : N2 - j2;
                const cx<T> u = grid[(size_t)j1 * P + colpos<N2, Q2, PADB>(j2)];
                const cx<T> um = grid[(size_t)n1 * P + colpos<N2, Q2, PADB>(n2)];
                uq[g] = mk<T>(u.x + um.x, u.y - um.y);
                if (hasb) uq2[g] = mk<T>(u.y + um.y, um.x - u.x);
            }
            __syncthreads();
        }
    }
}

template <typename TI, typename T, int N1, int N2, int Q1, int Q2, int NT, int PADB, bool GAM>
mb_status plane_launch(Problem* p, int ik, const void* c, void* u, int nbands, int ld, hipStream_t s) {
    const KPoint& kp = p->kp[ik];
    if (!kp.d_gtab || !p->d_Vt) return set_error(MB_ERR_INVALID_ARG, "plane kernel tables missing");
    if (kp.ng > 0 && (int)kp.rows.size() > N1) return set_error(MB_ERR_INVALID_ARG, "plane kernel: rows");
    constexpr bool dbl = sizeof(T) == 8;
    PlaneArgs<TI, T> a;
    a.c = (const cx<TI>*)c;
    a.u = (cx<T>*)u;
    a.bval = (const T*)(dbl ? (const void*)p->d_bval : (const void*)p->d_bvalf);
    a.Vt = (const T*)(dbl ? (const void*)p->d_Vt : (const void*)p->d_Vtf);
    a.gtab = kp.d_gtab;
    a.rows = kp.d_rows;
    a.tw1 = (const cx<T>*)(dbl ? p->d_tw1 : p->d_tw1f);
    a.tw2 = (const cx<T>*)(dbl ? p->d_tw2 : p->d_tw2f);
    a.nbands = GAM ? (nbands + 1) / 2 : nbands;
    a.nreal = nbands;
    a.ld = ld;
    a.nint = p->nint;
    a.nq = p->nq;
    a.nb = p->nb;
    a.nrows = (int)kp.rows.size();
    a.nzq = p->nzq;
    a.inv_n = (T)(1.0 / ((double)N1 * N2));
    constexpr size_t lds = plane_lds<T, N1, N2, Q2, PADB>();
    static_assert(lds <= 163840, "plane does not fit in LDS");
    auto kern = k_local_plane<TI, T, N1, N2, Q1, Q2, NT, PADB, GAM>;
    if (lds > 65536)
        MB_HIP_TRY(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const unsigned units = (unsigned)a.nbands * (unsigned)((p->nint + PLANE_NI - 1) / PLANE_NI);
    StageScope ts_(dbl ? MB_STAGE_LOCAL : MB_STAGE_LOCAL32, s, nbands);
    hipLaunchKernelGGL(kern, dim3(units), dim3(NT), lds, s, a);
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

template <typename TI, typename T, bool GAM>
mb_status plane_by_size(Problem* p, int ik, const void* c, void* u, int nbands, int ld, hipStream_t s) {
    // Two lane splits, 512 threads each (FP64 planes fill one CU's LDS, FP32 planes two
    // workgroups per CU): variant 0 holds 8 points per lane (16 lanes per 128-point
    // column, 8 per 64-point row; fewer registers), variant 1 holds 16 (8 and 4 lanes;
    // one lane-exchange stage less per line).  mb_autotune may pick either.
    constexpr int NT = 512;
    // untuned: on the 128 x 64 grid 16 points per lane in FP64 (26 ms against 44 ms per 320
    // bands of the surface slab), 8 in FP32 (13 ms against 18 ms); on the 36 x 36 grid 9
    // points per lane (FP64: 0.15 against 0.28 ms per 32 bands of the graphene-like slab)
    const KPoint::Tune& tn = p->kp[ik].tune[sizeof(T) == 8 ? 0 : (sizeof(TI) == 8 ? 2 : 1)];
    const int var = (tn.set && tn.kind == 3) ? tn.plane_var : (sizeof(T) == 8 && p->N1 == 128 ? 1 : 0);
    static_assert(64 * 16 % 16 == 0, "column tasks fill whole 16-lane rows");
    if (p->N1 == 128 && p->N2 == 64) {
        if (var == 1) return plane_launch<TI, T, 128, 64, 8, 4, NT, 1, GAM>(p, ik, c, u, nbands, ld, s);
        return plane_launch<TI, T, 128, 64, 16, 8, NT, 1, GAM>(p, ik, c, u, nbands, ld, s);
    }
    // 36 x 36 (the graphene-like slab): lines of 36 = 4 x 9 points over 4 lanes (144 line
    // tasks per pass, 192 threads) or 2 x 18 over 2 lanes (72 tasks, 128 threads); the
    // planes are small enough for several workgroups per CU
    if (p->N1 == 36 && p->N2 == 36) {
        if (var == 1) return plane_launch<TI, T, 36, 36, 2, 2, 128, 1, GAM>(p, ik, c, u, nbands, ld, s);
        return plane_launch<TI, T, 36, 36, 4, 4, 192, 1, GAM>(p, ik, c, u, nbands, ld, s);
    }
    return MB_ERR_INVALID_ARG;
}

// Electron density at the Gauss planes with the same lane-split transforms (the charge
// density of Sec. II.B.1): one workgroup per Gauss plane runs over the bands; per band
// the row pass evaluates and transforms the sphere rows into LDS and the column pass
// finishes the inverse transform, after which lane l of column j2 holds the points
// j1 = k + L1 bitrev(l) and adds w_b |psi|^2 / A to its accumulators.  Every thread owns
// the same grid points for all bands, so the sum over bands needs no atomics and runs in
// a fixed order.  FP64 arithmetic.
template <typename TI>
struct DensPlaneArgs {
    const cx<TI>* c;
    const double* w;
    double* rho;           // [q][j1][j2]
    const double* bval;
    const int32_t* gtab;
    const int32_t* rows;
    const cx<double>* tw1;
    const cx<double>* tw2;
    int nbands, ld, nq, nb, nrows, nzq;
    double inv_area;
};

template <typename TI, int N1, int N2, int Q1, int Q2, int NT, int PADB>
__global__ __launch_bounds__(NT) void k_density_plane(DensPlaneArgs<TI> a) {
    using T = double;
    constexpr int L1 = N1 / Q1, L2 = N2 / Q2;
    constexpr int P = plane_pitch<N2, Q2, PADB>();
    constexpr int CT = N2 * Q1 / NT;  // column tasks per thread
    static_assert(N2 * Q1 % NT == 0, "column tasks fill the workgroup");
    extern __shared__ unsigned char smem_raw[];
    cx<T>* tw1 = reinterpret_cast<cx<T>*>(smem_raw);
    cx<T>* tw2 = tw1 + N1;
    uint32_t* rmask = reinterpret_cast<uint32_t*>(tw2 + N2);
    cx<T>* grid = reinterpret_cast<cx<T>*>(smem_raw + plane_hdr<T, N1, N2>());
    const int q = (int)xcd_logical(blockIdx.x, gridDim.x);
    if (q >= a.nzq) return;
    const int s = q / a.nq;
    const int tid = threadIdx.x;
    for (int e = tid; e < N1; e += NT) tw1[e] = a.tw1[e];
    for (int e = tid; e < N2; e += NT) tw2[e] = a.tw2[e];
    for (int e = tid; e < (N1 + 31) / 32; e += NT) rmask[e] = 0u;
    __syncthreads();
    for (int e = tid; e < a.nrows; e += NT) {
        const int j1 = a.rows[e];
        atomicOr(&rmask[j1 >> 5], 1u << (j1 & 31));
    }
    __syncthreads();
    T bv[KORD];
#pragma unroll
    for (int t = 0; t < KORD; ++t) bv[t] = a.bval[(size_t)q * KORD + t];
    T acc[CT][L1];
#pragma unroll
    for (int c = 0; c < CT; ++c)
#pragma unroll
        for (int k = 0; k < L1; ++k) acc[c][k] = 0.0;
    const int nrt = (a.nrows * Q2 + 15) / 16 * 16;
    for (int b = 0; b < a.nbands; ++b) {
        const cx<TI>* cb = a.c + (size_t)b * a.nb * a.ld;
        // rows: evaluate on the sphere row, inverse transform along j2
        for (int task = tid; task < nrt; task += NT) {
            const int rc = (task >> 4) * (16 / Q2) + LaneMap<Q2>::line(task & 15);
            const int l = LaneMap<Q2>::lane(task & 15);
            if (rc >= a.nrows) continue;
            const int j1 = a.rows[rc];
            const int32_t* gr = a.gtab + (size_t)rc * N2;
            cx<T> x[L2];
            int gi[L2];
#pragma unroll
            for (int m = 0; m < L2; ++m) {
                gi[m] = gr[l + Q2 * m];
                x[m] = mk<T>(0, 0);
            }
#pragma unroll 1
            for (int t = 0; t < KORD; ++t) {
                const int row = s - 1 + t;
                if (row < 0 || row >= a.nb) continue;
                const cx<TI>* cr = cb + (size_t)row * a.ld;
#pragma unroll
                for (int m = 0; m < L2; ++m) {
                    const cx<TI> v = cr[gi[m] >= 0 ? gi[m] : 0];
                    const T w = gi[m] >= 0 ? bv[t] : (T)0;
                    x[m].x = fma(w, (T)v.x, x[m].x);
                    x[m].y = fma(w, (T)v.y, x[m].y);
                }
            }
            line_fft<T, L2, +1>(x);
#pragma unroll
            for (int k = 1; k < L2; ++k) x[k] = cmul(x[k], tw_at<T, +1>(tw2, l * k));
            dif_lanes<T, L2, Q2, N2, +1>(x, l, tw2);
            cx<T>* dst = grid + (size_t)j1 * P + colpos<N2, Q2, PADB>(L2 * bitrev_lane<Q2>(l));
#pragma unroll
            for (int k = 0; k < L2; ++k) dst[k] = x[k];
        }
        __syncthreads();
        // columns: inverse transform along j1, then |psi|^2 into the accumulators
        const T wb = a.w[b] * a.inv_area;
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int task = tid + c * NT;
            const int j2 = (task >> 4) * (16 / Q1) + LaneMap<Q1>::line(task & 15);
            const int l = LaneMap<Q1>::lane(task & 15);
            const int cp = colpos<N2, Q2, PADB>(j2);
            uint32_t live = 0u;
#pragma unroll
            for (int m = 0; m < L1; ++m) {
                const int j1 = l + Q1 * m;
                if ((rmask[j1 >> 5] >> (j1 & 31)) & 1u) live |= 1u << m;
            }
            cx<T> x[L1];
#pragma unroll
            for (int m = 0; m < L1; ++m) {
                const cx<T> v = grid[(size_t)(l + Q1 * m) * P + cp];
                x[m] = ((live >> m) & 1u) ? v : mk<T>(0, 0);
            }
            line_fft<T, L1, +1>(x);
#pragma unroll
            for (int k = 1; k < L1; ++k) x[k] = cmul(x[k], tw_at<T, +1>(tw1, l * k));
            dif_lanes<T, L1, Q1, N1, +1>(x, l, tw1);
#pragma unroll
            for (int k = 0; k < L1; ++k) acc[c][k] = fma(wb, x[k].x * x[k].x + x[k].y * x[k].y, acc[c][k]);
        }
        __syncthreads();  // the next band's row pass overwrites the plane
    }
    double* rq = a.rho + (size_t)q * N1 * N2;
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        const int task = tid + c * NT;
        const int j2 = (task >> 4) * (16 / Q1) + LaneMap<Q1>::line(task & 15);
        const int l = LaneMap<Q1>::lane(task & 15);
#pragma unroll
        for (int k = 0; k < L1; ++k) {
            const int j1 = k + L1 * bitrev_lane<Q1>(l);
            rq[(size_t)j1 * N2 + j2] += acc[c][k];
        }
    }
}

template <typename TI, int N1, int N2, int Q1, int Q2, int NT, int PADB>
mb_status density_plane_launch(Problem* p, int ik, const void* c, int nbands, int ld, const double* w, double* rho,
                               hipStream_t s) {
    const KPoint& kp = p->kp[ik];
    if (!kp.d_gtab) return set_error(MB_ERR_INVALID_ARG, "plane kernel tables missing");
    if (kp.ng > 0 && (int)kp.rows.size() > N1) return set_error(MB_ERR_INVALID_ARG, "plane kernel: rows");
    DensPlaneArgs<TI> a;
    a.c = (const cx<TI>*)c;
    a.w = w;
    a.rho = rho;
    a.bval = p->d_bval;
    a.gtab = kp.d_gtab;
    a.rows = kp.d_rows;
    a.tw1 = (const cx<double>*)p->d_tw1;
    a.tw2 = (const cx<double>*)p->d_tw2;
    a.nbands = nbands;
    a.ld = ld;
    a.nq = p->nq;
    a.nb = p->nb;
    a.nrows = (int)kp.rows.size();
    a.nzq = p->nzq;
    a.inv_area = 1.0 / p->area;
    constexpr size_t lds = plane_lds<double, N1, N2, Q2, PADB>();
    static_assert(lds <= 163840, "plane does not fit in LDS");
    auto kern = k_density_plane<TI, N1, N2, Q1, Q2, NT, PADB>;
    if (lds > 65536)
        MB_HIP_TRY(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    StageScope ts_(MB_STAGE_DENSITY, s, nbands);
    hipLaunchKernelGGL(kern, dim3((unsigned)p->nzq), dim3(NT), lds, s, a);
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

}  // namespace

bool plane_kernel_grid(const Problem* p) {
    return p->order == KORD && ((p->N1 == 128 && p->N2 == 64) || (p->N1 == 36 && p->N2 == 36));
}

// Returns MB_ERR_INVALID_ARG (no message) if the grid has no plane kernel.  FP64 planes
// with 16 points per lane (8 lanes per 128-point column, 4 per 64-point row).
mb_status launch_density_plane(Problem* p, int ik, const void* c, int nbands, int ld, const double* w, double* rho,
                               int prec, hipStream_t s) {
    if (p->order != KORD || p->N1 != 128 || p->N2 != 64) return MB_ERR_INVALID_ARG;
    if (nbands == 0) return MB_OK;
    if (prec == 0) return density_plane_launch<double, 128, 64, 8, 4, 512, 1>(p, ik, c, nbands, ld, w, rho, s);
    return density_plane_launch<float, 128, 64, 8, 4, 512, 1>(p, ik, c, nbands, ld, w, rho, s);
}

// Returns MB_ERR_INVALID_ARG (no message) if the grid has no plane kernel.
// gamma: real-wavefunction pairing (Gamma point, c(-G) = conj c(G) for every band).
mb_status launch_local_plane(Problem* p, int ik, const void* c, void* u, int nbands, int ld, int prec,
                             hipStream_t s, bool gamma) {
    if (!plane_kernel_grid(p)) return MB_ERR_INVALID_ARG;
    if (nbands == 0) return MB_OK;
    if (gamma) {
        if (prec == 0) return plane_by_size<double, double, true>(p, ik, c, u, nbands, ld, s);
        if (prec == 1) return plane_by_size<float, float, true>(p, ik, c, u, nbands, ld, s);
        return plane_by_size<double, float, true>(p, ik, c, u, nbands, ld, s);
    }
    if (prec == 0) return plane_by_size<double, double, false>(p, ik, c, u, nbands, ld, s);
    if (prec == 1) return plane_by_size<float, float, false>(p, ik, c, u, nbands, ld, s);
    return plane_by_size<double, float, false>(p, ik, c, u, nbands, ld, s);
}

namespace {
// Vt[q][j2][j1] = V[q][j1][j2]
template <typename T>
__global__ void k_vtranspose(const T* V, T* Vt, int N1, int N2, int nzq) {
    const size_t n = (size_t)N1 * N2 * nzq;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const size_t q = idx / ((size_t)N1 * N2);
    const int e = (int)(idx - q * N1 * N2);
    const int j2 = e / N1, j1 = e - j2 * N1;
    Vt[idx] = V[q * N1 * N2 + (size_t)j1 * N2 + j2];
}
}  // namespace

// Transposed copies of the potential (both precisions) for the plane kernel; allocated
// on first use, refreshed whenever the potential changes.
mb_status refresh_vt(Problem* p, hipStream_t s) {
    if (!plane_kernel_grid(p)) return MB_OK;
    const size_t n = (size_t)p->nzq * p->N1 * p->N2;
    if (!p->d_Vt && hipMalloc(&p->d_Vt, n * sizeof(double)) != hipSuccess)
        return set_error(MB_ERR_OOM, "transposed potential grid");
    if (!p->d_Vtf && hipMalloc(&p->d_Vtf, n * sizeof(float)) != hipSuccess)
        return set_error(MB_ERR_OOM, "transposed potential grid");
    const unsigned nblk = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_vtranspose<double>, dim3(nblk), dim3(256), 0, s, p->d_V, p->d_Vt, p->N1, p->N2, p->nzq);
    MB_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_vtranspose<float>, dim3(nblk), dim3(256), 0, s, p->d_Vf, p->d_Vtf, p->N1, p->N2, p->nzq);
    MB_HIP_TRY(hipGetLastError());
    MB_HIP_TRY(hipStreamSynchronize(s));
    return MB_OK;
}

}  // namespace mb
