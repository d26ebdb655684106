// Combine pass of H c for the plane layout of the local part, with both contractions
// along z on the matrix cores:
//   y(G, i) = 1/2 sum_j (D_z[i][j] + |k+G|^2 S_z[i][j]) c(G, j)        kinetic (banded)
//           + sum_q w_q B_i(z_q) u_q(G)                                 local part, planes q
//           + sum_p Z_p(i) F_p(G) P'_p                                  Kleinman-Bylander
//   sy(G, i) = sum_j S_z[i][j] c(G, j)                                  overlap (optional)
//            + sum_p Z_p(i) F_p(G) q_p <beta_p|c>                       ultrasoft term
// (kinetic, local and nonlocal matrix elements of Sec. II.B.1; P'_p = E_p <beta_p|c>;
// the ultrasoft term of Sec. II.B.2 only with augmentation charges).
// The last two terms are real (z) x complex (G) products C = A X with A[i][k] the
// spline weights w_q B_i(z_q) (k = plane q) or Z_p(i) (k = projector p) and
// X[k][G] = u_q(G) or F_p(G) P'_p, computed per 16-row x 16-column tile by
// v_mfma_f32_16x16x4_f32 / v_mfma_f64_16x16x4_f64 (real and imaginary parts of X as
// two products with the same A).  Only the planes of the intervals that hold the
// tile's splines and the projector groups whose z-window meets the tile enter.  The
// banded kinetic and overlap terms run on the vector units, in FP64, for the rows
// each lane holds in the matrix-core output layout.
// Lane layouts (gfx950): A[l%16][l/16], B[l/16][l%16]; output f32: D[4(l/16)+r][l%16],
// f64: D[4r + l/16][l%16], r < 4.
#include <algorithm>
#include <cstdlib>
#include <vector>

#include "cplx.h"
#include "mbks_internal.h"

namespace mb {

namespace {

constexpr int KORD = 4;

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <typename T>
struct MfmaAcc;
template <>
struct MfmaAcc<float> {
    using type = v4f;
    __device__ static v4f step(float a, float b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    // output row of accumulator element r for lane group g
    __device__ static int row(int g, int r) { return 4 * g + r; }
};
template <>
struct MfmaAcc<double> {
    using type = v4d;
    __device__ static v4d step(double a, double b, v4d c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int g, int r) { return 4 * r + g; }
};

template <typename TI, typename T>
struct ZArgs {
    const cx<TI>* c;       // [b][i][ld]
    const cx<T>* u;        // [b][q][ld] plane rows of the local part
    const T* wb;           // [q][kappa]: w_q B_{s-1+t}(z_q)
    const cx<T>* proj;     // [b][np]: E_p <beta_p|c> (null: no projectors)
    const cx<T>* projq;    // [b][np]: q_p <beta_p|c> (ultrasoft term of sy; AUG only)
    const cx<T>* F;        // [np][ld]
    const T* Z;            // [np][nb]
    const int32_t* gwin;   // [ngrp][2]: union z-window of each group of 16 projectors
    cx<TI>* y;
    cx<TI>* sy;            // may be null
    const double* sband;
    const double* dband;
    const double* kg2;
    int nbands, ld, ng, nb, nint, nq, nzq, np;
};

// One workgroup = 4 waves = 4 consecutive 16-column tiles of one 16-row tile, for
// ZC_BB bands.  AUG: sy also takes the projector expansion of projq.
template <typename TI, typename T, bool AUG, int ZC_BB>
__global__ __launch_bounds__(256) void k_zcombine(ZArgs<TI, T> a) {
    using A = MfmaAcc<T>;
    using V = typename A::type;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int G0 = ((int)blockIdx.x * 4 + wave) * 16;
    if (G0 >= a.ld) return;
    const int i0 = (int)blockIdx.y * 16;
    const int b0 = (int)blockIdx.z * ZC_BB;
    const int nbg = min(ZC_BB, a.nbands - b0);
    const int Gm = G0 + m;
    const bool gv = Gm < a.ng;
    const int ia = i0 + m;  // row of this lane's A operand

    V acc[ZC_BB][2];
    constexpr int BQ = AUG ? ZC_BB : 1;
    V accq[BQ][2];
#pragma unroll
    for (int bb = 0; bb < ZC_BB; ++bb)
#pragma unroll
        for (int h = 0; h < 2; ++h) acc[bb][h] = V{0, 0, 0, 0};
#pragma unroll
    for (int bb = 0; bb < BQ; ++bb)
#pragma unroll
        for (int h = 0; h < 2; ++h) accq[bb][h] = V{0, 0, 0, 0};

    // Band rows of the loads are clamped into the call's bands and columns into the
    // row stride: lanes past N_G (padding) and bands past nbands load valid memory whose
    // products only reach outputs that are never written (padding columns get zeros).
    int brow[ZC_BB];
#pragma unroll
    for (int bb = 0; bb < ZC_BB; ++bb) brow[bb] = min(b0 + bb, a.nbands - 1);
    const int Gl = gv ? Gm : 0;
    // local part: planes of the intervals s = i - 2 .. i + 1 of the tile's rows, four
    // planes per step (lane group g takes plane qk + g); the next step's operands are
    // loaded before the current step's products are issued
    {
        const int s_lo = max(i0 - 2, 0), s_hi = min(i0 + 16, a.nint - 1);
        const int q_lo = s_lo * a.nq, q_hi = (s_hi + 1) * a.nq;
        int q = q_lo + g;
        int sq = q / a.nq, rq = q - sq * a.nq;  // interval and Gauss point of plane q
        auto weight = [&](int qq, int ss) -> T {
            if (qq >= q_hi || ia >= a.nb) return (T)0;
            const int t = ia + 1 - ss;
            return (t >= 0 && t < KORD) ? a.wb[(size_t)qq * KORD + t] : (T)0;
        };
        auto load = [&](int qq, cx<T>* v) {
            const int qc = qq < q_hi ? qq : q_lo;
#pragma unroll
            for (int bb = 0; bb < ZC_BB; ++bb) v[bb] = a.u[((size_t)brow[bb] * a.nzq + qc) * a.ld + Gl];
        };
        cx<T> vn[ZC_BB];
        T wn = weight(q, sq);
        load(q, vn);
        for (int qk = q_lo; qk < q_hi; qk += 4) {
            cx<T> v[ZC_BB];
#pragma unroll
            for (int bb = 0; bb < ZC_BB; ++bb) v[bb] = vn[bb];
            const T w = wn;
            q += 4;
            rq += 4;
            while (rq >= a.nq) { rq -= a.nq; ++sq; }
            if (qk + 4 < q_hi) {
                wn = weight(q, sq);
                load(q, vn);
            }
#pragma unroll
            for (int bb = 0; bb < ZC_BB; ++bb) {
                acc[bb][0] = A::step(w, v[bb].x, acc[bb][0]);
                acc[bb][1] = A::step(w, v[bb].y, acc[bb][1]);
            }
        }
    }
    // Kleinman-Bylander expansion: projector groups whose window meets the tile
    if (a.proj) {
        const int ngrp = (a.np + 15) / 16;
        for (int grp = 0; grp < ngrp; ++grp) {
            if (a.gwin[2 * grp] > i0 + 15 || a.gwin[2 * grp + 1] < i0) continue;
            T z[4];
            cx<T> f[4], pp[4][ZC_BB], pq[4][BQ];
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const int p = grp * 16 + 4 * st + g;
                const int pc = min(p, a.np - 1);
                z[st] = (p < a.np && ia < a.nb) ? a.Z[(size_t)pc * a.nb + ia] : (T)0;
                f[st] = a.F[(size_t)pc * a.ld + Gl];
#pragma unroll
                for (int bb = 0; bb < ZC_BB; ++bb) pp[st][bb] = a.proj[(size_t)brow[bb] * a.np + pc];
                if constexpr (AUG) {
#pragma unroll
                    for (int bb = 0; bb < ZC_BB; ++bb) pq[st][bb] = a.projq[(size_t)brow[bb] * a.np + pc];
                }
            }
#pragma unroll
            for (int st = 0; st < 4; ++st) {
#pragma unroll
                for (int bb = 0; bb < ZC_BB; ++bb) {
                    const cx<T> v = cmul(f[st], pp[st][bb]);
                    acc[bb][0] = A::step(z[st], v.x, acc[bb][0]);
                    acc[bb][1] = A::step(z[st], v.y, acc[bb][1]);
                }
                if constexpr (AUG) {
#pragma unroll
                    for (int bb = 0; bb < ZC_BB; ++bb) {
                        const cx<T> v = cmul(f[st], pq[st][bb]);
                        accq[bb][0] = A::step(z[st], v.x, accq[bb][0]);
                        accq[bb][1] = A::step(z[st], v.y, accq[bb][1]);
                    }
                }
            }
        }
    }
    if (Gm >= a.ld) return;
    // Banded kinetic and overlap sums and the stores.  Every load takes a clamped, valid
    // index and out-of-range terms are masked afterwards, so that no load sits under a
    // lane-dependent branch (the compiler waits for every load in flight where such
    // branches join, which would serialize the c-row and band loads)
    const int Gc = gv ? Gm : 0;
    const double kk = gv ? 0.5 * a.kg2[Gc] : 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = i0 + A::row(g, r);
        const bool rowok = i < a.nb;
        const int ic = rowok ? i : a.nb - 1;
        double sv[2 * KORD - 1], tv[2 * KORD - 1];
        int jr[2 * KORD - 1];
#pragma unroll
        for (int d = -(KORD - 1); d <= KORD - 1; ++d) {
            const int j = ic + d;
            const bool ok = j >= 0 && j < a.nb;
            const int jc = ok ? j : ic;
            const int lo = d >= 0 ? ic : jc;
            const int dd = d >= 0 ? d : -d;
            const double s0 = a.sband[lo * KORD + dd];
            const double d0 = a.dband[lo * KORD + dd];
            sv[d + KORD - 1] = ok ? s0 : 0.0;
            tv[d + KORD - 1] = ok ? 0.5 * d0 : 0.0;
            jr[d + KORD - 1] = jc;
        }
#pragma unroll
        for (int bb = 0; bb < ZC_BB; ++bb) {
            if (bb >= nbg) break;
            const size_t vb = (size_t)(b0 + bb) * a.nb * a.ld;
            double sr = 0, si = 0, tr = 0, ti = 0;
#pragma unroll
            for (int e = 0; e < 2 * KORD - 1; ++e) {
                const cx<TI> cv = a.c[vb + (size_t)jr[e] * a.ld + Gc];
                sr += sv[e] * (double)cv.x;
                si += sv[e] * (double)cv.y;
                tr += tv[e] * (double)cv.x;
                ti += tv[e] * (double)cv.y;
            }
            double qr = 0.0, qi = 0.0;
            if constexpr (AUG) {
                qr = (double)accq[bb][0][r];
                qi = (double)accq[bb][1][r];
            }
            const double yr = tr + kk * sr + (double)acc[bb][0][r];
            const double yi = ti + kk * si + (double)acc[bb][1][r];
            if (rowok) {
                // padding columns (G >= N_G) get zeros
                a.y[vb + (size_t)i * a.ld + Gm] = gv ? mk<TI>((TI)yr, (TI)yi) : mk<TI>(0, 0);
                if (a.sy) a.sy[vb + (size_t)i * a.ld + Gm] = gv ? mk<TI>((TI)(sr + qr), (TI)(si + qi)) : mk<TI>(0, 0);
            }
        }
    }
}

template <typename TI, typename T>
mb_status zcombine_impl(Problem* p, int ik, const void* c, const void* u, const void* proj, void* y, void* sy,
                        int nbands, int ld, hipStream_t s, const void* projq) {
    const KPoint& kp = p->kp[ik];
    constexpr bool dbl = sizeof(T) == 8;
    ZArgs<TI, T> a;
    a.c = (const cx<TI>*)c;
    a.u = (const cx<T>*)u;
    a.wb = (const T*)(dbl ? (const void*)p->d_wbval : (const void*)p->d_wbvalf);
    a.proj = p->np > 0 ? (const cx<T>*)proj : nullptr;
    a.projq = p->np > 0 && sy ? (const cx<T>*)projq : nullptr;
    if (a.projq && !a.proj) return set_error(MB_ERR_INVALID_ARG, "zcombine: ultrasoft term without projections");
    a.F = (const cx<T>*)(dbl ? kp.d_F64 : kp.d_F32);
    a.Z = (const T*)(dbl ? (const void*)p->d_Z : (const void*)p->d_Zf);
    a.gwin = p->d_gwin;
    a.y = (cx<TI>*)y;
    a.sy = (cx<TI>*)sy;
    a.sband = p->d_sband;
    a.dband = p->d_dband;
    a.kg2 = kp.d_kg2;
    a.nbands = nbands;
    a.ld = ld;
    a.ng = kp.ng;
    a.nb = p->nb;
    a.nint = p->nint;
    a.nq = p->nq;
    a.nzq = p->nzq;
    a.np = p->np;
    if (p->np > 0 && !p->d_gwin) return set_error(MB_ERR_INVALID_ARG, "projector group windows not uploaded");
    // bands per wave: 2 (MBKS_ZC_BANDS=1, 4 or 8 selects 1, 4 or 8).  Measured on the
    // 128x64 surface slab, 320 bands: FP64 9.3 ms with 2 against 11.9 (4) and 18.7 (8);
    // FP32 5.9 against 6.1 and 6.8 (more waves per SIMD hide the plane-row loads better)
    const char* zb = getenv("MBKS_ZC_BANDS");
    const int bbz = zb && zb[0] == '8' ? 8 : zb && zb[0] == '4' ? 4 : zb && zb[0] == '1' ? 1 : 2;
    const dim3 grid((unsigned)((ld + 63) / 64), (unsigned)((p->nb + 15) / 16), (unsigned)((nbands + bbz - 1) / bbz));
    StageScope ts_(MB_STAGE_COMBINE, s, nbands);
    if (bbz == 8) {
        if (a.projq)
            hipLaunchKernelGGL((k_zcombine<TI, T, true, 8>), grid, dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_zcombine<TI, T, false, 8>), grid, dim3(256), 0, s, a);
    } else if (bbz == 4) {
        if (a.projq)
            hipLaunchKernelGGL((k_zcombine<TI, T, true, 4>), grid, dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_zcombine<TI, T, false, 4>), grid, dim3(256), 0, s, a);
    } else if (bbz == 1) {
        if (a.projq)
            hipLaunchKernelGGL((k_zcombine<TI, T, true, 1>), grid, dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_zcombine<TI, T, false, 1>), grid, dim3(256), 0, s, a);
    } else {
        if (a.projq)
            hipLaunchKernelGGL((k_zcombine<TI, T, true, 2>), grid, dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_zcombine<TI, T, false, 2>), grid, dim3(256), 0, s, a);
    }
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

}  // namespace

// y = H c from the plane rows u of the local part (sy = S c if non-null); prec as
// launch_combine
mb_status launch_zcombine(Problem* p, int ik, const void* c, const void* u, const void* proj, void* y, void* sy,
                          int nbands, int ld, int prec, hipStream_t s, const void* projq) {
    if (nbands == 0) return MB_OK;
    if (prec == 0) return zcombine_impl<double, double>(p, ik, c, u, proj, y, sy, nbands, ld, s, projq);
    if (prec == 1) return zcombine_impl<float, float>(p, ik, c, u, proj, y, sy, nbands, ld, s, projq);
    return zcombine_impl<double, float>(p, ik, c, u, proj, y, sy, nbands, ld, s, projq);
}

}  // namespace mb
