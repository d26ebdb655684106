// Kleinman-Bylander projections on the matrix cores (eq. KBeq and its matrix
// elements, Sec. II.B.1):
//   proj[b][p] = E_p sum_i Z_p(i) sum_G conj(F_p(G)) c_b(G, i)
// One wave computes, for one spline row i, a 16 (projectors) x 16 (bands) tile
// of sum_G conj(F_p(G)) c_b(G, i) with MFMA instructions and scales it by
// Z_p(i); a second kernel sums the row partials in a fixed order and applies E_p.
// The complex product is four real products:
//   re = Fr cr + Fi ci,  im = Fr ci - Fi cr.
// Variants: FP32 operands on v_mfma_f32_16x16x4_f32, and BF16x3, where every
// FP32 operand x is split into hi = bf16(x), lo = bf16(x - hi) and each real
// product is hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16 (FP32
// accumulation; about 16 significant bits per product).
// Lane layouts (checked on gfx950): 16x16x4 f32: lane l holds A[l%16][l/16] and
// B[l/16][l%16]; 16x16x32 bf16: A[l%16][8(l/16)+t], B[8(l/16)+t][l%16], t < 8;
// both: D[4(l/16)+r][l%16], r < 4.  The order of the k sum inside a step is free,
// so lane group g = l/16 takes the contiguous k range of its step.
#include <algorithm>
#include <cstdlib>
#include <vector>

#include "cplx.h"
#include "mbks_internal.h"

namespace mb {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

template <typename TI>
__device__ inline cx<float> ldc(const cx<TI>* p) {
    cx<TI> v = *p;
    return mk<float>((float)v.x, (float)v.y);
}

// partial[i][p][b] = Z_p(i) sum_G conj(F_p(G)) c_b(G, i), FP32 MFMA
template <typename TI>
__global__ __launch_bounds__(64) void k_nlproj_f32(const cx<TI>* c, const cx<float>* F, const float* Z,
                                                   const int32_t* gwin, cx<float>* partial, int nbands, int np,
                                                   int ng, int nb, int ld, int npad, int nbpad) {
    const int i = blockIdx.x;
    const int b0 = blockIdx.y * 16;
    const int grp = blockIdx.z;
    if (i < gwin[2 * grp] || i > gwin[2 * grp + 1]) return;
    const int lane = threadIdx.x;
    const int m = lane % 16, g = lane / 16;
    const int p = grp * 16 + m;
    const int b = b0 + m;
    // rows of projectors past np and bands past nbands are clamped: their products only
    // reach padding entries of the partial sums; columns past N_G are zero (the padding
    // of the vectors is not read)
    const cx<float>* Fp = F + (size_t)min(p, np - 1) * ld;
    const cx<TI>* cb = c + ((size_t)min(b, nbands - 1) * nb + i) * ld;
    v4f accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
    // this lane group's 4 consecutive k of a 16-wide chunk; the next chunk is loaded
    // before the current chunk's products are issued
    auto load = [&](int k0, cx<float>* fa, cx<float>* cv) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = k0 + 4 * g + s;
            const bool in = k < ng;
            const int kc = in ? k : 0;
            const cx<float> fv = Fp[kc], v = ldc<TI>(cb + kc);
            fa[s] = in ? fv : mk<float>(0, 0);
            cv[s] = in ? v : mk<float>(0, 0);
        }
    };
    cx<float> fn[4], cn[4];
    load(0, fn, cn);
    for (int k0 = 0; k0 < ng; k0 += 16) {
        cx<float> fa[4], cv[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) { fa[s] = fn[s]; cv[s] = cn[s]; }
        if (k0 + 16 < ng) load(k0 + 16, fn, cn);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            accr = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[s].x, cv[s].x, accr, 0, 0, 0);
            accr = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[s].y, cv[s].y, accr, 0, 0, 0);
            acci = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[s].x, cv[s].y, acci, 0, 0, 0);
            acci = __builtin_amdgcn_mfma_f32_16x16x4f32(-fa[s].y, cv[s].x, acci, 0, 0, 0);
        }
    }
    // D[4g + r][m]: projector row 4g + r of the group, band column m
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int pr = grp * 16 + 4 * g + r;
        const float z = pr < np ? Z[(size_t)pr * nb + i] : 0.0f;
        partial[((size_t)i * npad + pr) * nbpad + b0 + m] = mk<float>(z * accr[r], z * acci[r]);
    }
}

// The same FP32 partials with up to MG projector groups per wave: the groups are the
// ones whose z window holds the wave's spline row (slot blockIdx.z * MG + j of the row's
// list), so the row's 16 band chunks are loaded once per k step and multiplied into the
// accumulators of every group instead of once per group (on the 128x64 surface slab a row
// lies in the windows of 7.4 groups on average).  Each group's products are issued in the
// same order as in k_nlproj_f32, so the partials are the same.
template <typename TI, int MG>
__global__ __launch_bounds__(64) void k_nlproj_f32m(const cx<TI>* c, const cx<float>* F, const float* Z,
                                                    const int32_t* rgoff, const int32_t* rglist,
                                                    cx<float>* partial, int nbands, int np, int ng, int nb, int ld,
                                                    int npad, int nbpad) {
    const int i = blockIdx.x;
    const int b0 = blockIdx.y * 16;
    const int s0 = rgoff[i] + blockIdx.z * MG;
    const int nslot = min(MG, rgoff[i + 1] - s0);
    if (nslot <= 0) return;
    const int lane = threadIdx.x;
    const int m = lane % 16, g = lane / 16;
    const int b = b0 + m;
    const cx<TI>* cb = c + ((size_t)min(b, nbands - 1) * nb + i) * ld;
    int grp[MG];
    const cx<float>* Fp[MG];
    v4f accr[MG], acci[MG];
#pragma unroll
    for (int j = 0; j < MG; ++j) {
        grp[j] = j < nslot ? rglist[s0 + j] : 0;
        Fp[j] = F + (size_t)min(grp[j] * 16 + m, np - 1) * ld;
        accr[j] = v4f{0, 0, 0, 0};
        acci[j] = v4f{0, 0, 0, 0};
    }
    for (int k0 = 0; k0 < ng; k0 += 16) {
        cx<float> cv[4];
        bool in[4];
        int kc[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = k0 + 4 * g + s;
            in[s] = k < ng;
            kc[s] = in[s] ? k : 0;
            const cx<float> v = ldc<TI>(cb + kc[s]);
            cv[s] = in[s] ? v : mk<float>(0, 0);
        }
#pragma unroll
        for (int j = 0; j < MG; ++j) {
            if (j >= nslot) break;
            cx<float> fa[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const cx<float> fv = Fp[j][kc[s]];
                fa[s] = in[s] ? fv : mk<float>(0, 0);
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                accr[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[s].x, cv[s].x, accr[j], 0, 0, 0);
                accr[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[s].y, cv[s].y, accr[j], 0, 0, 0);
                acci[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[s].x, cv[s].y, acci[j], 0, 0, 0);
                acci[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(-fa[s].y, cv[s].x, acci[j], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < MG; ++j) {
        if (j >= nslot) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int pr = grp[j] * 16 + 4 * g + r;
            const float z = pr < np ? Z[(size_t)pr * nb + i] : 0.0f;
            partial[((size_t)i * npad + pr) * nbpad + b0 + m] = mk<float>(z * accr[j][r], z * acci[j][r]);
        }
    }
}

// the same partials in FP64 on v_mfma_f64_16x16x4_f64, whose output layout differs:
// lane l holds D[4r + l/16][l%16] (checked on gfx950)
typedef double v4d __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(64) void k_nlproj_f64(const cx<double>* c, const cx<double>* F, const double* Z,
                                                   const int32_t* gwin, cx<double>* partial, int nbands, int np,
                                                   int ng, int nb, int ld, int npad, int nbpad) {
    const int i = blockIdx.x;
    const int b0 = blockIdx.y * 16;
    const int grp = blockIdx.z;
    if (i < gwin[2 * grp] || i > gwin[2 * grp + 1]) return;
    const int lane = threadIdx.x;
    const int m = lane % 16, g = lane / 16;
    const int p = grp * 16 + m;
    const int b = b0 + m;
    const cx<double>* Fp = F + (size_t)min(p, np - 1) * ld;
    const cx<double>* cb = c + ((size_t)min(b, nbands - 1) * nb + i) * ld;
    v4d accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
    auto load = [&](int k0, cx<double>* fa, cx<double>* cv) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = k0 + 4 * g + s;
            const bool in = k < ng;
            const int kc = in ? k : 0;
            const cx<double> fv = Fp[kc], v = cb[kc];
            fa[s] = in ? fv : mk<double>(0, 0);
            cv[s] = in ? v : mk<double>(0, 0);
        }
    };
    cx<double> fn[4], cn[4];
    load(0, fn, cn);
    for (int k0 = 0; k0 < ng; k0 += 16) {
        cx<double> fa[4], cv[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) { fa[s] = fn[s]; cv[s] = cn[s]; }
        if (k0 + 16 < ng) load(k0 + 16, fn, cn);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            accr = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s].x, cv[s].x, accr, 0, 0, 0);
            accr = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s].y, cv[s].y, accr, 0, 0, 0);
            acci = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s].x, cv[s].y, acci, 0, 0, 0);
            acci = __builtin_amdgcn_mfma_f64_16x16x4f64(-fa[s].y, cv[s].x, acci, 0, 0, 0);
        }
    }
    // D[4r + g][m]: projector row 4r + g of the group, band column m
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int pr = grp * 16 + 4 * r + g;
        const double z = pr < np ? Z[(size_t)pr * nb + i] : 0.0;
        partial[((size_t)i * npad + pr) * nbpad + b0 + m] = mk<double>(z * accr[r], z * acci[r]);
    }
}

// FP64 partials with up to MG projector groups per wave (as k_nlproj_f32m); the FP64
// output layout D[4r + l/16][l%16]
template <int MG>
__global__ __launch_bounds__(64) void k_nlproj_f64m(const cx<double>* c, const cx<double>* F, const double* Z,
                                                    const int32_t* rgoff, const int32_t* rglist,
                                                    cx<double>* partial, int nbands, int np, int ng, int nb, int ld,
                                                    int npad, int nbpad) {
    const int i = blockIdx.x;
    const int b0 = blockIdx.y * 16;
    const int s0 = rgoff[i] + blockIdx.z * MG;
    const int nslot = min(MG, rgoff[i + 1] - s0);
    if (nslot <= 0) return;
    const int lane = threadIdx.x;
    const int m = lane % 16, g = lane / 16;
    const int b = b0 + m;
    const cx<double>* cb = c + ((size_t)min(b, nbands - 1) * nb + i) * ld;
    int grp[MG];
    const cx<double>* Fp[MG];
    v4d accr[MG], acci[MG];
#pragma unroll
    for (int j = 0; j < MG; ++j) {
        grp[j] = j < nslot ? rglist[s0 + j] : 0;
        Fp[j] = F + (size_t)min(grp[j] * 16 + m, np - 1) * ld;
        accr[j] = v4d{0, 0, 0, 0};
        acci[j] = v4d{0, 0, 0, 0};
    }
    for (int k0 = 0; k0 < ng; k0 += 16) {
        cx<double> cv[4];
        bool in[4];
        int kc[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = k0 + 4 * g + s;
            in[s] = k < ng;
            kc[s] = in[s] ? k : 0;
            const cx<double> v = cb[kc[s]];
            cv[s] = in[s] ? v : mk<double>(0, 0);
        }
#pragma unroll
        for (int j = 0; j < MG; ++j) {
            if (j >= nslot) break;
            cx<double> fa[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const cx<double> fv = Fp[j][kc[s]];
                fa[s] = in[s] ? fv : mk<double>(0, 0);
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                accr[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s].x, cv[s].x, accr[j], 0, 0, 0);
                accr[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s].y, cv[s].y, accr[j], 0, 0, 0);
                acci[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[s].x, cv[s].y, acci[j], 0, 0, 0);
                acci[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-fa[s].y, cv[s].x, acci[j], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < MG; ++j) {
        if (j >= nslot) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int pr = grp[j] * 16 + 4 * r + g;
            const double z = pr < np ? Z[(size_t)pr * nb + i] : 0.0;
            partial[((size_t)i * npad + pr) * nbpad + b0 + m] = mk<double>(z * accr[j][r], z * acci[j][r]);
        }
    }
}

__device__ inline void split_bf16(float x, __bf16& hi, __bf16& lo) {
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}

// same partials, BF16x3 on v_mfma_f32_16x16x32_bf16
template <typename TI>
__global__ __launch_bounds__(64) void k_nlproj_bf16x3(const cx<TI>* c, const cx<float>* F, const float* Z,
                                                      const int32_t* gwin, cx<float>* partial, int nbands, int np,
                                                      int ng, int nb, int ld, int npad, int nbpad) {
    const int i = blockIdx.x;
    const int b0 = blockIdx.y * 16;
    const int grp = blockIdx.z;
    if (i < gwin[2 * grp] || i > gwin[2 * grp + 1]) return;
    const int lane = threadIdx.x;
    const int m = lane % 16, g = lane / 16;
    const int p = grp * 16 + m;
    const int b = b0 + m;
    const cx<float>* Fp = F + (size_t)min(p, np - 1) * ld;
    const cx<TI>* cb = c + ((size_t)min(b, nbands - 1) * nb + i) * ld;
    const bool pv = p < np, bv = b < nbands;
    v4f accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
    for (int k0 = 0; k0 < ng; k0 += 32) {
        v8bf frh, frl, fih, fil, fin_h, fin_l, crh, crl, cih, cil;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int k = k0 + 8 * g + t;
            const bool in = k < ng;
            const cx<float> f = (pv && in) ? Fp[k] : mk<float>(0, 0);
            const cx<float> v = (bv && in) ? ldc<TI>(cb + k) : mk<float>(0, 0);
            __bf16 h, l;
            split_bf16(f.x, h, l); frh[t] = h; frl[t] = l;
            split_bf16(f.y, h, l); fih[t] = h; fil[t] = l;
            split_bf16(-f.y, h, l); fin_h[t] = h; fin_l[t] = l;
            split_bf16(v.x, h, l); crh[t] = h; crl[t] = l;
            split_bf16(v.y, h, l); cih[t] = h; cil[t] = l;
        }
        // re += Fr cr + Fi ci ; im += Fr ci - Fi cr ; each as hi*hi + hi*lo + lo*hi
        accr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frh, crh, accr, 0, 0, 0);
        accr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frh, crl, accr, 0, 0, 0);
        accr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frl, crh, accr, 0, 0, 0);
        accr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fih, cih, accr, 0, 0, 0);
        accr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fih, cil, accr, 0, 0, 0);
        accr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fil, cih, accr, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frh, cih, acci, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frh, cil, acci, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frl, cih, acci, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fin_h, crh, acci, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fin_h, crl, acci, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fin_l, crh, acci, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int pr = grp * 16 + 4 * g + r;
        const float z = pr < np ? Z[(size_t)pr * nb + i] : 0.0f;
        partial[((size_t)i * npad + pr) * nbpad + b0 + m] = mk<float>(z * accr[r], z * acci[r]);
    }
}

// proj[b][p] = E_p sum_{i in group window} partial[i][p][b] (fixed order over i), and
// projq[b][p] = Q_p times the same sum when projq is given (ultrasoft overlap)
__global__ void k_nlproj_reduce(const cx<float>* partial, const int32_t* gwin, const float* E, cx<float>* proj,
                                const float* Q, cx<float>* projq, int nbands, int np, int npad, int nbpad) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nbands * np) return;
    const int b = idx / np, p = idx % np;
    const int grp = p / 16;
    const int lo = gwin[2 * grp], hi = gwin[2 * grp + 1];
    float re = 0.f, im = 0.f;
    for (int i = lo; i <= hi; ++i) {
        cx<float> v = partial[((size_t)i * npad + p) * nbpad + b];
        re += v.x;
        im += v.y;
    }
    proj[(size_t)b * np + p] = mk<float>(E[p] * re, E[p] * im);
    if (projq) projq[(size_t)b * np + p] = mk<float>(Q[p] * re, Q[p] * im);
}

// FP64 form of the reduction (energies E_p in FP64)
__global__ void k_nlproj_reduce64(const cx<double>* partial, const int32_t* gwin, const double* E, cx<double>* proj,
                                  const double* Q, cx<double>* projq, int nbands, int np, int npad, int nbpad) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nbands * np) return;
    const int b = idx / np, p = idx % np;
    const int grp = p / 16;
    const int lo = gwin[2 * grp], hi = gwin[2 * grp + 1];
    double re = 0.0, im = 0.0;
    for (int i = lo; i <= hi; ++i) {
        cx<double> v = partial[((size_t)i * npad + p) * nbpad + b];
        re += v.x;
        im += v.y;
    }
    proj[(size_t)b * np + p] = mk<double>(E[p] * re, E[p] * im);
    if (projq) projq[(size_t)b * np + p] = mk<double>(Q[p] * re, Q[p] * im);
}

}  // namespace

// mode 0: FP64 MFMA (complex128 vectors), mode 1: FP32 MFMA, mode 2: BF16x3 MFMA;
// vin64: vectors are complex128
// union z-window of every group of 16 projectors (set-up, once per problem)
mb_status upload_group_windows(Problem* p) {
    const int ngrp = (p->np + 15) / 16;
    std::vector<int32_t> gw(2 * ngrp);
    for (int gi = 0; gi < ngrp; ++gi) {
        int lo = p->nb, hi = -1;
        for (int q = gi * 16; q < std::min(p->np, gi * 16 + 16); ++q) {
            if (p->zwin[2 * q + 1] < p->zwin[2 * q]) continue;
            lo = std::min(lo, (int)p->zwin[2 * q]);
            hi = std::max(hi, (int)p->zwin[2 * q + 1]);
        }
        if (hi < 0) { lo = 0; hi = -1; }
        gw[2 * gi] = lo;
        gw[2 * gi + 1] = hi;
    }
    MB_HIP_TRY(hipMalloc(&p->d_gwin, gw.size() * sizeof(int32_t)));
    MB_HIP_TRY(hipMemcpy(p->d_gwin, gw.data(), gw.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    std::vector<int32_t> off(p->nb + 1, 0), list;
    p->rg_max = 0;
    for (int i = 0; i < p->nb; ++i) {
        off[i] = (int32_t)list.size();
        for (int gi = 0; gi < ngrp; ++gi)
            if (gw[2 * gi] <= i && i <= gw[2 * gi + 1]) list.push_back(gi);
        p->rg_max = std::max(p->rg_max, (int)list.size() - off[i]);
    }
    off[p->nb] = (int32_t)list.size();
    if (list.empty()) list.push_back(0);
    MB_HIP_TRY(hipMalloc(&p->d_rgoff, off.size() * sizeof(int32_t)));
    MB_HIP_TRY(hipMemcpy(p->d_rgoff, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    MB_HIP_TRY(hipMalloc(&p->d_rglist, list.size() * sizeof(int32_t)));
    MB_HIP_TRY(hipMemcpy(p->d_rglist, list.data(), list.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    return MB_OK;
}

size_t nl_mfma_part_bytes(const Problem* p, int nbands, int mode) {
    const int npad = (p->np + 15) / 16 * 16;
    const int nbpad = (nbands + 15) / 16 * 16;
    return (size_t)p->nb * npad * nbpad * (mode == 0 ? sizeof(cx<double>) : sizeof(cx<float>));
}

mb_status launch_nl_project_mfma(Problem* p, int ik, const void* c, void* proj, int nbands, int ld, int mode,
                                 bool vin64, hipStream_t s, void* nlpart, int scale, void* projq) {
    if (p->np == 0) return MB_OK;
    const KPoint& kp = p->kp[ik];
    const int ngrp = (p->np + 15) / 16;
    const int npad = ngrp * 16;
    const int nbpad = (nbands + 15) / 16 * 16;
    if (!p->d_gwin) return set_error(MB_ERR_INVALID_ARG, "projector group windows not uploaded");
    KPoint& kw = p->kp[ik];
    if (!nlpart) {
        mb_status st = ensure_hws(kw, kw.ws_nlpart, nl_mfma_part_bytes(p, nbands, mode));
        if (st != MB_OK) return st;
        nlpart = kw.ws_nlpart.ptr;
    }
    StageScope ts_(MB_STAGE_NL_PROJECT, s, nbands);
    dim3 grid(p->nb, nbpad / 16, ngrp);
    const char* multi_env = getenv("MBKS_NL_MULTI");
    const bool multi = !(multi_env && multi_env[0] == '0') && p->d_rgoff && p->rg_max > 1;
    constexpr int MG = 4;  // projector groups per wave (MBKS_NL_MULTI=0: one)
    const dim3 gm(p->nb, nbpad / 16, (std::max(p->rg_max, 1) + MG - 1) / MG);
    if (mode == 0) {
        cx<double>* part64 = (cx<double>*)nlpart;
        if (multi)
            hipLaunchKernelGGL(k_nlproj_f64m<MG>, gm, dim3(64), 0, s, (const cx<double>*)c,
                               (const cx<double>*)kp.d_F64, p->d_Z, p->d_rgoff, p->d_rglist, part64, nbands, p->np,
                               kp.ng, p->nb, ld, npad, nbpad);
        else
            hipLaunchKernelGGL(k_nlproj_f64, grid, dim3(64), 0, s, (const cx<double>*)c, (const cx<double>*)kp.d_F64,
                               p->d_Z, p->d_gwin, part64, nbands, p->np, kp.ng, p->nb, ld, npad, nbpad);
        MB_HIP_TRY(hipGetLastError());
        const int tot = nbands * p->np;
        const double* sc = scale == PROJ_Q ? p->d_Q : scale == PROJ_ONE ? p->d_one : p->d_E;
        hipLaunchKernelGGL(k_nlproj_reduce64, dim3((tot + 255) / 256), dim3(256), 0, s, part64, p->d_gwin, sc,
                           (cx<double>*)proj, p->d_Q, (cx<double>*)projq, nbands, p->np, npad, nbpad);
        MB_HIP_TRY(hipGetLastError());
        return MB_OK;
    }
    cx<float>* part = (cx<float>*)nlpart;
    const cx<float>* F = (const cx<float>*)kp.d_F32;
    if (mode == 1 && multi) {
        if (vin64)
            hipLaunchKernelGGL((k_nlproj_f32m<double, MG>), gm, dim3(64), 0, s, (const cx<double>*)c, F, p->d_Zf,
                               p->d_rgoff, p->d_rglist, part, nbands, p->np, kp.ng, p->nb, ld, npad, nbpad);
        else
            hipLaunchKernelGGL((k_nlproj_f32m<float, MG>), gm, dim3(64), 0, s, (const cx<float>*)c, F, p->d_Zf,
                               p->d_rgoff, p->d_rglist, part, nbands, p->np, kp.ng, p->nb, ld, npad, nbpad);
    } else if (mode == 1) {
        if (vin64)
            hipLaunchKernelGGL(k_nlproj_f32<double>, grid, dim3(64), 0, s, (const cx<double>*)c, F, p->d_Zf,
                               p->d_gwin, part, nbands, p->np, kp.ng, p->nb, ld, npad, nbpad);
        else
            hipLaunchKernelGGL(k_nlproj_f32<float>, grid, dim3(64), 0, s, (const cx<float>*)c, F, p->d_Zf,
                               p->d_gwin, part, nbands, p->np, kp.ng, p->nb, ld, npad, nbpad);
    } else {
        if (vin64)
            hipLaunchKernelGGL(k_nlproj_bf16x3<double>, grid, dim3(64), 0, s, (const cx<double>*)c, F, p->d_Zf,
                               p->d_gwin, part, nbands, p->np, kp.ng, p->nb, ld, npad, nbpad);
        else
            hipLaunchKernelGGL(k_nlproj_bf16x3<float>, grid, dim3(64), 0, s, (const cx<float>*)c, F, p->d_Zf,
                               p->d_gwin, part, nbands, p->np, kp.ng, p->nb, ld, npad, nbpad);
    }
    MB_HIP_TRY(hipGetLastError());
    const int tot = nbands * p->np;
    const float* scf = scale == PROJ_Q ? p->d_Qf : scale == PROJ_ONE ? p->d_onef : p->d_Ef;
    hipLaunchKernelGGL(k_nlproj_reduce, dim3((tot + 255) / 256), dim3(256), 0, s, part, p->d_gwin, scf,
                       (cx<float>*)proj, p->d_Qf, (cx<float>*)projq, nbands, p->np, npad, nbpad);
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

}  // namespace mb
