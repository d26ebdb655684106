// FP64 dense kernels of the eigensolver (Sec. II.C): Gram matrices in the S
// inner product, linear combinations of vectors, batched dot products, and the
// projected generalized eigenproblems solved by Cholesky reduction and the
// cyclic Jacobi method.  Vectors are addressed through device tables of
// pointers so one launch serves every block of the block cycle.
#include <cmath>
#include <cstdlib>
#include <string>

#include "cplx.h"
#include "dense.h"
#include "mbks_internal.h"

namespace mb {

namespace {

using zc = cx<double>;

// ---------------------------------------------------------------------------
// Gram: C_z[m][n] = sum_k conj(A_{z,m}[k]) B_{z,n}[k], split over k chunks.
// part[z][chunk][m][n]; reduced in fixed order by k_gram_reduce.
// ---------------------------------------------------------------------------
constexpr int GT = 16;   // output tile
constexpr int GK = 32;   // k per LDS stage

__global__ __launch_bounds__(256) void k_gram(const zc* const* ta, const zc* const* tb, int MA, int NB, int64_t K,
                                              int64_t kchunk, int nchunk, int tiles_n, zc* part) {
    __shared__ zc As[GT][GK + 1];
    __shared__ zc Bs[GT][GK + 1];
    const int z = blockIdx.z;
    const int chunk = blockIdx.x;
    const int tm = blockIdx.y / tiles_n, tn = blockIdx.y % tiles_n;
    const int tx = threadIdx.x % GT, ty = threadIdx.x / GT;  // ty -> m, tx -> n
    const int m0 = tm * GT, n0 = tn * GT;
    const int64_t k0 = (int64_t)chunk * kchunk;
    const int64_t k1 = min(K, k0 + kchunk);
    zc acc = mk<double>(0, 0);
    for (int64_t kb = k0; kb < k1; kb += GK) {
        // 256 threads load 16 x 32 of A and of B
        for (int e = threadIdx.x; e < GT * GK; e += 256) {
            int r = e / GK, kk = e % GK;
            int64_t k = kb + kk;
            zc va = mk<double>(0, 0), vb = mk<double>(0, 0);
            if (k < k1) {
                if (m0 + r < MA) va = ta[(size_t)z * MA + m0 + r][k];
                if (n0 + r < NB) vb = tb[(size_t)z * NB + n0 + r][k];
            }
            As[r][kk] = va;
            Bs[r][kk] = vb;
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < GK; ++kk) cfmac(acc, As[ty][kk], Bs[tx][kk]);
        __syncthreads();
    }
    const int m = m0 + ty, n = n0 + tx;
    if (m < MA && n < NB) part[(((size_t)z * nchunk + chunk) * MA + m) * NB + n] = acc;
}

// the same product with 32 x 32 output tiles, each thread holding a 2 x 2 block of
// outputs (m = m0 + ty + 16 a, n = n0 + tx + 16 c): one LDS read per complex FMA
constexpr int GT2 = 32;
constexpr int GK2 = 16;

__global__ __launch_bounds__(256) void k_gram32(const zc* const* ta, const zc* const* tb, int MA, int NB, int64_t K,
                                                int64_t kchunk, int nchunk, int tiles_n, zc* part) {
    __shared__ zc As[GT2][GK2 + 1];
    __shared__ zc Bs[GT2][GK2 + 1];
    const int z = blockIdx.z;
    const int chunk = blockIdx.x;
    const int tm = blockIdx.y / tiles_n, tn = blockIdx.y % tiles_n;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int m0 = tm * GT2, n0 = tn * GT2;
    const int64_t k0 = (int64_t)chunk * kchunk;
    const int64_t k1 = min(K, k0 + kchunk);
    zc acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[a][c] = mk<double>(0, 0);
    for (int64_t kb = k0; kb < k1; kb += GK2) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = threadIdx.x + 256 * u;
            const int r = e / GK2, kk = e % GK2;
            const int64_t k = kb + kk;
            zc va = mk<double>(0, 0), vb = mk<double>(0, 0);
            if (k < k1) {
                if (m0 + r < MA) va = ta[(size_t)z * MA + m0 + r][k];
                if (n0 + r < NB) vb = tb[(size_t)z * NB + n0 + r][k];
            }
            As[r][kk] = va;
            Bs[r][kk] = vb;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < GK2; ++kk) {
            const zc a0 = As[ty][kk], a1 = As[ty + 16][kk];
            const zc b0 = Bs[tx][kk], b1 = Bs[tx + 16][kk];
            cfmac(acc[0][0], a0, b0);
            cfmac(acc[0][1], a0, b1);
            cfmac(acc[1][0], a1, b0);
            cfmac(acc[1][1], a1, b1);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int m = m0 + ty + 16 * a, n = n0 + tx + 16 * c;
            if (m < MA && n < NB) part[(((size_t)z * nchunk + chunk) * MA + m) * NB + n] = acc[a][c];
        }
}

// the widest products (MA, NB >= 256): 64 x 64 output tiles, each thread a 4 x 4
// block (m = m0 + ty + 16 a, n = n0 + tx + 16 c), so 8 LDS reads feed 16 complex
// FMAs; the next k step's tile is loaded into registers while the current one is
// used.  Blocks run tile-fastest through (tile, chunk, z), mapped so that each XCD
// takes a contiguous run: the tiles of one k chunk share that XCD's L2.
constexpr int G64 = 64;
constexpr int GK64 = 16;

__global__ __launch_bounds__(256) void k_gram64(const zc* const* ta, const zc* const* tb, int MA, int NB, int64_t K,
                                                int64_t kchunk, int nchunk, int tiles_m, int tiles_n, zc* part) {
    __shared__ zc As[G64][GK64 + 1];
    __shared__ zc Bs[G64][GK64 + 1];
    const unsigned L = xcd_logical(blockIdx.x, gridDim.x);
    const int ntile = tiles_m * tiles_n;
    const int tile = (int)(L % ntile);
    const int chunk = (int)((L / ntile) % nchunk);
    const int z = (int)(L / ntile / nchunk);
    const int tm = tile / tiles_n, tn = tile % tiles_n;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int m0 = tm * G64, n0 = tn * G64;
    const int64_t k0 = (int64_t)chunk * kchunk;
    const int64_t k1 = min(K, k0 + kchunk);
    // loader mapping: element e = tid + 256 u of the 64 x 16 tile, row e / 16, k e % 16
    const int lk = threadIdx.x % GK64, lr = threadIdx.x / GK64;  // rows lr + 16 u
    const zc* arow[4];
    const zc* brow[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int r = lr + 16 * u;
        arow[u] = m0 + r < MA ? ta[(size_t)z * MA + m0 + r] : nullptr;
        brow[u] = n0 + r < NB ? tb[(size_t)z * NB + n0 + r] : nullptr;
    }
    zc pa[4], pb[4];
    auto fetch = [&](int64_t kb) {
        const int64_t k = kb + lk;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            pa[u] = (k < k1 && arow[u]) ? arow[u][k] : mk<double>(0, 0);
            pb[u] = (k < k1 && brow[u]) ? brow[u][k] : mk<double>(0, 0);
        }
    };
    zc acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = mk<double>(0, 0);
    if (k0 < k1) fetch(k0);
    for (int64_t kb = k0; kb < k1; kb += GK64) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            As[lr + 16 * u][lk] = pa[u];
            Bs[lr + 16 * u][lk] = pb[u];
        }
        __syncthreads();
        if (kb + GK64 < k1) fetch(kb + GK64);
#pragma unroll 2
        for (int kk = 0; kk < GK64; ++kk) {
            zc a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = As[ty + 16 * i][kk];
                b[i] = Bs[tx + 16 * i][kk];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int c = 0; c < 4; ++c) cfmac(acc[i][c], a[i], b[c]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int m = m0 + ty + 16 * a, n = n0 + tx + 16 * c;
            if (m < MA && n < NB) part[(((size_t)z * nchunk + chunk) * MA + m) * NB + n] = acc[a][c];
        }
}

// The same 64 x 64 tiles on the FP64 matrix cores (v_mfma_f64_16x16x4_f64): each wave
// owns a 32 x 32 quarter of the tile as 2 x 2 MFMA tiles.  With a = A_m[k], b = B_n[k],
//   Re sum conj(a) b = sum a.x b.x + sum a.y b.y,  Im = sum a.x b.y + sum (-a.y) b.x,
// four real 16x16x4 products per tile and k step.  Lane layout of the instruction
// (checked on gfx950): lane l supplies A[l%16][l/16] and B[l/16][l%16] and holds
// D[4r + l/16][l%16], r < 4 (unlike the FP32 16x16x4 form, whose D rows are 4(l/16) + r).
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

// herm != 0 (MA == NB, Hermitian result): only the tiles with tm <= tn are computed
// (tiles_m (tiles_m + 1) / 2 of them); k_gram_reduce fills the others by conjugation.
__global__ __launch_bounds__(256) void k_gram_mfma(const zc* const* ta, const zc* const* tb, int MA, int NB,
                                                   int64_t K, int64_t kchunk, int nchunk, int tiles_m, int tiles_n,
                                                   zc* part, int herm) {
    __shared__ zc As[G64][GK64 + 1];
    __shared__ zc Bs[G64][GK64 + 1];
    const unsigned L = xcd_logical(blockIdx.x, gridDim.x);
    const int ntile = herm ? tiles_m * (tiles_m + 1) / 2 : tiles_m * tiles_n;
    const int tile = (int)(L % ntile);
    const int chunk = (int)((L / ntile) % nchunk);
    const int z = (int)(L / ntile / nchunk);
    int tm = tile / tiles_n, tn = tile % tiles_n;
    if (herm) {
        // row tm of the upper triangle holds tiles_m - tm tiles
        tm = 0;
        int rem = tile;
        while (rem >= tiles_m - tm) {
            rem -= tiles_m - tm;
            ++tm;
        }
        tn = tm + rem;
    }
    const int m0 = tm * G64, n0 = tn * G64;
    const int64_t k0 = (int64_t)chunk * kchunk;
    const int64_t k1 = min(K, k0 + kchunk);
    const int lk = threadIdx.x % GK64, lr = threadIdx.x / GK64;  // loader: rows lr + 16 u, column lk
    const zc* arow[4];
    const zc* brow[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int r = lr + 16 * u;
        arow[u] = m0 + r < MA ? ta[(size_t)z * MA + m0 + r] : nullptr;
        brow[u] = n0 + r < NB ? tb[(size_t)z * NB + n0 + r] : nullptr;
    }
    zc pa[4], pb[4];
    auto fetch = [&](int64_t kb) {
        const int64_t k = kb + lk;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            pa[u] = (k < k1 && arow[u]) ? arow[u][k] : mk<double>(0, 0);
            pb[u] = (k < k1 && brow[u]) ? brow[u][k] : mk<double>(0, 0);
        }
    };
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int wr = (wave / 2) * 32, wc = (wave % 2) * 32;  // this wave's quarter of the tile
    const int li = lane % 16, lg = lane / 16;
    mfma_d4 cr[2][2], ci[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            cr[a][c] = mfma_d4{0.0, 0.0, 0.0, 0.0};
            ci[a][c] = mfma_d4{0.0, 0.0, 0.0, 0.0};
        }
    if (k0 < k1) fetch(k0);
    for (int64_t kb = k0; kb < k1; kb += GK64) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            As[lr + 16 * u][lk] = pa[u];
            Bs[lr + 16 * u][lk] = pb[u];
        }
        __syncthreads();
        if (kb + GK64 < k1) fetch(kb + GK64);
#pragma unroll
        for (int st = 0; st < GK64 / 4; ++st) {
            const int kk = 4 * st + lg;
            zc av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = As[wr + 16 * a + li][kk];
#pragma unroll
            for (int c = 0; c < 2; ++c) bv[c] = Bs[wc + 16 * c + li][kk];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    cr[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].x, bv[c].x, cr[a][c], 0, 0, 0);
                    cr[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].y, bv[c].y, cr[a][c], 0, 0, 0);
                    ci[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].x, bv[c].y, ci[a][c], 0, 0, 0);
                    ci[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[a].y, bv[c].x, ci[a][c], 0, 0, 0);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wr + 16 * a + 4 * r + lg, n = n0 + wc + 16 * c + li;
                if (m < MA && n < NB)
                    part[(((size_t)z * nchunk + chunk) * MA + m) * NB + n] = mk<double>(cr[a][c][r], ci[a][c][r]);
            }
}

typedef float mfma_f4 __attribute__((ext_vector_type(4)));

// narrow products (MA <= 16): block (chunk, n, z) streams its k range once, each
// thread accumulating conj(A_m[k]) B_n[k] for every m in registers; wave shuffles
// and one LDS pass reduce the block's MA sums into part[z][chunk][m][n]
constexpr int SKINNY = 16;

__global__ __launch_bounds__(256) void k_gram_skinny(const zc* const* ta, const zc* const* tb, int MA, int NB,
                                                     int64_t K, int64_t kchunk, int nchunk, zc* part) {
    const int z = blockIdx.z;
    const int n = blockIdx.y;
    const int chunk = blockIdx.x;
    const int64_t k0 = (int64_t)chunk * kchunk;
    const int64_t k1 = min(K, k0 + kchunk);
    const zc* bcol = tb[(size_t)z * NB + n];
    const zc* const* arow = ta + (size_t)z * MA;
    zc acc[SKINNY];
#pragma unroll
    for (int m = 0; m < SKINNY; ++m) acc[m] = mk<double>(0, 0);
    for (int64_t k = k0 + threadIdx.x; k < k1; k += 256) {
        const zc bv = bcol[k];
#pragma unroll
        for (int m = 0; m < SKINNY; ++m)
            if (m < MA) cfmac(acc[m], arow[m][k], bv);
    }
    __shared__ zc red[4][SKINNY];
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
#pragma unroll
    for (int m = 0; m < SKINNY; ++m) {
        if (m < MA) {
            double re = acc[m].x, im = acc[m].y;
            for (int off = 32; off > 0; off >>= 1) {
                re += __shfl_down(re, off, 64);
                im += __shfl_down(im, off, 64);
            }
            if (lane == 0) red[wave][m] = mk<double>(re, im);
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < MA) {
        const int m = threadIdx.x;
        zc v = red[0][m];
        for (int w = 1; w < 4; ++w) v = cadd(v, red[w][m]);
        part[(((size_t)z * nchunk + chunk) * MA + m) * NB + n] = v;
    }
}

// small square-ish products (MA, NB <= 6, e.g. the per-block projected matrices):
// block (chunk, z) streams every A_m and B_n of its k range exactly once and keeps
// all MA x NB sums in registers
constexpr int TINY = 6;

__global__ __launch_bounds__(256) void k_gram_tiny(const zc* const* ta, const zc* const* tb, int MA, int NB,
                                                   int64_t K, int64_t kchunk, int nchunk, zc* part) {
    const int z = blockIdx.z;
    const int chunk = blockIdx.x;
    const int64_t k0 = (int64_t)chunk * kchunk;
    const int64_t k1 = min(K, k0 + kchunk);
    const zc* A[TINY];
    const zc* B[TINY];
#pragma unroll
    for (int m = 0; m < TINY; ++m) {
        A[m] = m < MA ? ta[(size_t)z * MA + m] : nullptr;
        B[m] = m < NB ? tb[(size_t)z * NB + m] : nullptr;
    }
    zc acc[TINY][TINY];
#pragma unroll
    for (int m = 0; m < TINY; ++m)
#pragma unroll
        for (int n = 0; n < TINY; ++n) acc[m][n] = mk<double>(0, 0);
    for (int64_t k = k0 + threadIdx.x; k < k1; k += 256) {
        zc av[TINY], bv[TINY];
#pragma unroll
        for (int m = 0; m < TINY; ++m) {
            av[m] = m < MA ? A[m][k] : mk<double>(0, 0);
            bv[m] = m < NB ? B[m][k] : mk<double>(0, 0);
        }
#pragma unroll
        for (int m = 0; m < TINY; ++m)
#pragma unroll
            for (int n = 0; n < TINY; ++n)
                if (m < MA && n < NB) cfmac(acc[m][n], av[m], bv[n]);
    }
    __shared__ zc red[4][TINY * TINY];
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
#pragma unroll
    for (int m = 0; m < TINY; ++m)
#pragma unroll
        for (int n = 0; n < TINY; ++n) {
            if (m < MA && n < NB) {
                double re = acc[m][n].x, im = acc[m][n].y;
                for (int off = 32; off > 0; off >>= 1) {
                    re += __shfl_down(re, off, 64);
                    im += __shfl_down(im, off, 64);
                }
                if (lane == 0) red[wave][m * TINY + n] = mk<double>(re, im);
            }
        }
    __syncthreads();
    if ((int)threadIdx.x < MA * NB) {
        const int m = threadIdx.x / NB, n = threadIdx.x % NB;
        zc v = red[0][m * TINY + n];
        for (int w = 1; w < 4; ++w) v = cadd(v, red[w][m * TINY + n]);
        part[(((size_t)z * nchunk + chunk) * MA + m) * NB + n] = v;
    }
}

// one wave per output element: lanes stride over the chunks, then a shuffle tree
// htile > 0: Hermitian product computed on the tiles (of htile rows) with tm <= tn only;
// an element of a lower tile is the conjugate of its mirror
__global__ __launch_bounds__(256) void k_gram_reduce(const zc* part, zc* out, int MA, int NB, int nchunk, int nz,
                                                     int htile) {
    const size_t per = (size_t)MA * NB;
    const size_t idx = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int lane = threadIdx.x % 64;
    if (idx >= per * nz) return;
    const size_t z = idx / per;
    size_t e = idx % per;
    bool mirror = false;
    if (htile > 0) {
        const int m = (int)(e / NB), n = (int)(e % NB);
        if (m / htile > n / htile) {
            e = (size_t)n * NB + m;
            mirror = true;
        }
    }
    double re = 0.0, im = 0.0;
    for (int c = lane; c < nchunk; c += 64) {
        zc v = part[(z * nchunk + c) * per + e];
        re += v.x;
        im += v.y;
    }
    for (int off = 32; off > 0; off >>= 1) {
        re += __shfl_down(re, off, 64);
        im += __shfl_down(im, off, 64);
    }
    if (lane == 0) out[idx] = mk<double>(re, mirror ? -im : im);
}

// ---------------------------------------------------------------------------
// Combination: Y_{z,n}[k] = alpha * sum_m W_z[m][n] X_{z,m}[k] + beta * Y_{z,n}[k]
// ---------------------------------------------------------------------------
// One thread per k and CW outputs.  The coefficients are read straight from global
// memory at wave-uniform addresses (they compile to scalar loads into SGPRs, which
// the FMAs take as operands), so there is no LDS staging and no limit on MI; each
// input element is read once per CW outputs.  Inputs are
// loaded through global-address-space pointers: flat loads would share the scalar
// loads' wait counter, and every coefficient wait would then drain them.
typedef double gd2 __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(1))) gd2* gd2p;

template <int CW, bool FULL>
__global__ __launch_bounds__(256) void k_combo_w(const zc* const* __restrict__ tx, zc* const* __restrict__ ty,
                                                 const zc* __restrict__ W, int MI, int NO, int64_t K, double alpha,
                                                 double beta, int nbeg) {
    const int z = blockIdx.z;
    const int n0 = nbeg + blockIdx.y * CW;
    const int nn = FULL ? CW : NO - n0;
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= K) return;
    const zc* __restrict__ Wz = W + (size_t)z * MI * NO + n0;
    const zc* const* xt = tx + (size_t)z * MI;
    zc acc[CW];
#pragma unroll
    for (int j = 0; j < CW; ++j) acc[j] = mk<double>(0, 0);
#pragma unroll 2
    for (int m = 0; m < MI; ++m) {
        const gd2 xv = ((gd2p)xt[m])[k];
        const zc x = mk<double>(xv.x, xv.y);
        const zc* __restrict__ wr = Wz + (size_t)m * NO;
#pragma unroll
        for (int j = 0; j < CW; ++j)
            if (FULL || j < nn) cfma(acc[j], wr[j], x);
    }
#pragma unroll
    for (int j = 0; j < CW; ++j) {
        if (FULL || j < nn) {
            zc* yp = ty[(size_t)z * NO + n0 + j] + k;
            zc o = cscale(acc[j], alpha);
            if (beta != 0.0) o = cadd(o, cscale(*yp, beta));
            *yp = o;
        }
    }
}

// The wide combinations on the FP64 matrix cores (v_mfma_f64_16x16x4_f64): Y = X W as a
// product of a K x MI block of vectors with the MI x NO coefficients.  A workgroup owns
// 64 consecutive k (16 per wave) and 64 outputs (the output groups of one k range are
// consecutive blocks on one XCD, so the later groups re-read X from L2); the
// coefficients of each chunk of 16 inputs are staged in LDS once for the four waves
// (two buffers: the next chunk's operands load while the current chunk's products issue),
// and each lane loads one element of X per 4 inputs (lane l: input m0 + l/16,
// k = k0 + l%16, so 16 lanes read 256 contiguous bytes of one vector).  Complex
// products as four real ones per tile:
//   Re += Xr Wr + (-Xi) Wi,  Im += Xr Wi + Xi Wr.
// Output of tile t in lane l: rows (k) 4r + l/16, column (output) 16t + l%16; the tiles
// go through LDS so that every output vector is written (and, with beta, read) as 64
// consecutive k, 1 KB per instruction, instead of 64-byte pieces of 16 vectors.
constexpr int CM_K = 64, CM_N = 64, CM_M = 16, CM_H = 32;  // CM_H: outputs per epilogue pass
constexpr size_t CM_LDS = sizeof(zc) * (CM_K * (CM_H + 1) > 2 * CM_M * (CM_N + 1) ? CM_K * (CM_H + 1)
                                                                                    : 2 * CM_M * (CM_N + 1));

__global__ __launch_bounds__(256) void k_combo_mfma(const zc* const* __restrict__ tx, zc* const* __restrict__ ty,
                                                    const zc* __restrict__ W, int MI, int NO, int64_t K,
                                                    double alpha, double beta, int nng, int64_t nkb) {
    __shared__ __attribute__((aligned(16))) unsigned char smem[CM_LDS];
    zc (*Ws)[CM_N + 1] = reinterpret_cast<zc (*)[CM_N + 1]>(smem);
    zc (*Os)[CM_H + 1] = reinterpret_cast<zc (*)[CM_H + 1]>(smem);
    const unsigned L = xcd_logical(blockIdx.x, gridDim.x);
    const int z = blockIdx.y;
    const int ng = (int)(L % (unsigned)nng);
    const int64_t kb = (int64_t)(L / (unsigned)nng);
    if (kb >= nkb) return;
    const int n0 = ng * CM_N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int64_t k0 = kb * CM_K;
    const int64_t ka = k0 + wave * 16 + li;  // row of this lane's A operand
    const bool kok = ka < K;
    const zc* const* xt = tx + (size_t)z * MI;
    const zc* Wz = W + (size_t)z * MI * NO;
    mfma_d4 cr[CM_N / 16], ci[CM_N / 16];
#pragma unroll
    for (int t = 0; t < CM_N / 16; ++t) {
        cr[t] = mfma_d4{0.0, 0.0, 0.0, 0.0};
        ci[t] = mfma_d4{0.0, 0.0, 0.0, 0.0};
    }
    // operands of one chunk of CM_M inputs: this lane's X elements for the chunk's four
    // steps and this thread's share of the chunk's coefficients; the next chunk's are
    // loaded while the current chunk's products issue (two coefficient buffers in LDS)
    constexpr int WPT = CM_M * CM_N / 256;
    zc av[CM_M / 4], wv[WPT];
    auto load = [&](int m0) {
#pragma unroll
        for (int st = 0; st < CM_M / 4; ++st) {
            const int m = m0 + 4 * st + lg;
            av[st] = (kok && m < MI) ? xt[m][ka] : mk<double>(0, 0);
        }
#pragma unroll
        for (int u = 0; u < WPT; ++u) {
            const int e = threadIdx.x + 256 * u;
            const int m = m0 + e / CM_N, n = n0 + e % CM_N;
            wv[u] = (m < MI && n < NO) ? Wz[(size_t)m * NO + n] : mk<double>(0, 0);
        }
    };
    auto stage = [&](int buf) {
#pragma unroll
        for (int u = 0; u < WPT; ++u) {
            const int e = threadIdx.x + 256 * u;
            Ws[buf * CM_M + e / CM_N][e % CM_N] = wv[u];
        }
    };
    load(0);
    stage(0);
    __syncthreads();
    int buf = 0;
    for (int m0 = 0; m0 < MI; m0 += CM_M) {
        zc a[CM_M / 4];
#pragma unroll
        for (int st = 0; st < CM_M / 4; ++st) a[st] = av[st];
        const bool more = m0 + CM_M < MI;
        if (more) load(m0 + CM_M);
#pragma unroll
        for (int st = 0; st < CM_M / 4; ++st) {
            const double xr = a[st].x, xi = a[st].y;
#pragma unroll
            for (int t = 0; t < CM_N / 16; ++t) {
                const zc w = Ws[buf * CM_M + 4 * st + lg][16 * t + li];
                cr[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr, w.x, cr[t], 0, 0, 0);
                cr[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(-xi, w.y, cr[t], 0, 0, 0);
                ci[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr, w.y, ci[t], 0, 0, 0);
                ci[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(xi, w.x, ci[t], 0, 0, 0);
            }
        }
        if (more) stage(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    // epilogue in two passes of CM_H outputs: tiles to LDS as [k][n], then each wave
    // writes CM_H / 4 outputs, lane l taking row k0 + l
#pragma unroll
    for (int h = 0; h < CM_N / CM_H; ++h) {
#pragma unroll
        for (int tt = 0; tt < CM_H / 16; ++tt) {
            const int t = h * (CM_H / 16) + tt;
#pragma unroll
            for (int r = 0; r < 4; ++r) Os[wave * 16 + 4 * r + lg][16 * tt + li] = mk<double>(cr[t][r], ci[t][r]);
        }
        __syncthreads();
        const int64_t k = k0 + lane;
#pragma unroll
        for (int j = 0; j < CM_H / 4; ++j) {
            const int nn = wave * (CM_H / 4) + j;
            const int n = n0 + h * CM_H + nn;
            if (n < NO && k < K) {
                zc* yv = ty[(size_t)z * NO + n];
                const zc v = Os[lane][nn];
                zc o = mk<double>(alpha * v.x, alpha * v.y);
                if (beta != 0.0) o = cadd(o, cscale(yv[k], beta));
                yv[k] = o;
            }
        }
        __syncthreads();
    }
}

// The combination with FP32 matrix-core arithmetic on FP64 vectors (reduced-precision
// cycles of the eigensolver): the same tiles and staging as k_combo_mfma, operands
// converted to FP32 on load, products accumulated in FP32, outputs (and beta Y) in FP64.
__global__ __launch_bounds__(256) void k_combo_mfma32(const zc* const* __restrict__ tx, zc* const* __restrict__ ty,
                                                      const zc* __restrict__ W, int MI, int NO, int64_t K,
                                                      double alpha, double beta, int nng, int64_t nkb) {
    __shared__ __attribute__((aligned(16))) unsigned char smem[CM_LDS];
    cx<float> (*Ws)[CM_N + 1] = reinterpret_cast<cx<float> (*)[CM_N + 1]>(smem);
    zc (*Os)[CM_H + 1] = reinterpret_cast<zc (*)[CM_H + 1]>(smem);
    const unsigned L = xcd_logical(blockIdx.x, gridDim.x);
    const int z = blockIdx.y;
    const int ng = (int)(L % (unsigned)nng);
    const int64_t kb = (int64_t)(L / (unsigned)nng);
    if (kb >= nkb) return;
    const int n0 = ng * CM_N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int64_t k0 = kb * CM_K;
    const int64_t ka = k0 + wave * 16 + li;
    const bool kok = ka < K;
    const zc* const* xt = tx + (size_t)z * MI;
    const zc* Wz = W + (size_t)z * MI * NO;
    mfma_f4 cr[CM_N / 16], ci[CM_N / 16];
#pragma unroll
    for (int t = 0; t < CM_N / 16; ++t) {
        cr[t] = mfma_f4{0.f, 0.f, 0.f, 0.f};
        ci[t] = mfma_f4{0.f, 0.f, 0.f, 0.f};
    }
    constexpr int WPT = CM_M * CM_N / 256;
    cx<float> av[CM_M / 4], wv[WPT];
    auto load = [&](int m0) {
#pragma unroll
        for (int st = 0; st < CM_M / 4; ++st) {
            const int m = m0 + 4 * st + lg;
            const zc v = (kok && m < MI) ? xt[m][ka] : mk<double>(0, 0);
            av[st] = mk<float>((float)v.x, (float)v.y);
        }
#pragma unroll
        for (int u = 0; u < WPT; ++u) {
            const int e = threadIdx.x + 256 * u;
            const int m = m0 + e / CM_N, n = n0 + e % CM_N;
            const zc v = (m < MI && n < NO) ? Wz[(size_t)m * NO + n] : mk<double>(0, 0);
            wv[u] = mk<float>((float)v.x, (float)v.y);
        }
    };
    auto stage = [&](int buf) {
#pragma unroll
        for (int u = 0; u < WPT; ++u) {
            const int e = threadIdx.x + 256 * u;
            Ws[buf * CM_M + e / CM_N][e % CM_N] = wv[u];
        }
    };
    load(0);
    stage(0);
    __syncthreads();
    int buf = 0;
    for (int m0 = 0; m0 < MI; m0 += CM_M) {
        cx<float> a[CM_M / 4];
#pragma unroll
        for (int st = 0; st < CM_M / 4; ++st) a[st] = av[st];
        const bool more = m0 + CM_M < MI;
        if (more) load(m0 + CM_M);
#pragma unroll
        for (int st = 0; st < CM_M / 4; ++st) {
            const float xr = a[st].x, xi = a[st].y;
#pragma unroll
            for (int t = 0; t < CM_N / 16; ++t) {
                const cx<float> w = Ws[buf * CM_M + 4 * st + lg][16 * t + li];
                cr[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xr, w.x, cr[t], 0, 0, 0);
                cr[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(-xi, w.y, cr[t], 0, 0, 0);
                ci[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xr, w.y, ci[t], 0, 0, 0);
                ci[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xi, w.x, ci[t], 0, 0, 0);
            }
        }
        if (more) stage(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int h = 0; h < CM_N / CM_H; ++h) {
#pragma unroll
        for (int tt = 0; tt < CM_H / 16; ++tt) {
            const int t = h * (CM_H / 16) + tt;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                Os[wave * 16 + 4 * lg + r][16 * tt + li] = mk<double>((double)cr[t][r], (double)ci[t][r]);
        }
        __syncthreads();
        const int64_t k = k0 + lane;
#pragma unroll
        for (int j = 0; j < CM_H / 4; ++j) {
            const int nn = wave * (CM_H / 4) + j;
            const int n = n0 + h * CM_H + nn;
            if (n < NO && k < K) {
                zc* yv = ty[(size_t)z * NO + n];
                const zc v = Os[lane][nn];
                zc o = mk<double>(alpha * v.x, alpha * v.y);
                if (beta != 0.0) o = cadd(o, cscale(yv[k], beta));
                yv[k] = o;
            }
        }
        __syncthreads();
    }
}

template <int CW>
void launch_combo_w(const void* const* tx, void* const* ty, const void* W, int MI, int NO, int nz, int64_t K,
                    double alpha, double beta, hipStream_t s) {
    const unsigned kb = (unsigned)((K + 255) / 256);
    const int nfull = NO / CW;
    if (nfull > 0)
        hipLaunchKernelGGL((k_combo_w<CW, true>), dim3(kb, nfull, nz), dim3(256), 0, s, (const zc* const*)tx,
                           (zc* const*)ty, (const zc*)W, MI, NO, K, alpha, beta, 0);
    if (NO % CW)
        hipLaunchKernelGGL((k_combo_w<CW, false>), dim3(kb, 1, nz), dim3(256), 0, s, (const zc* const*)tx,
                           (zc* const*)ty, (const zc*)W, MI, NO, K, alpha, beta, nfull * CW);
}

// ---------------------------------------------------------------------------
// batched dots d_v = sum_k conj(A_v[k]) B_v[k], split over k chunks; partials
// part[v][chunk] reduced in fixed order by k_dots_reduce
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_dots(const zc* const* ta, const zc* const* tb, int64_t K, int64_t kchunk,
                                              int nchunk, zc* part) {
    const int v = blockIdx.y;
    const int c = blockIdx.x;
    const zc* a = ta[v];
    const zc* b = tb[v];
    const int64_t k0 = (int64_t)c * kchunk, k1 = min(K, k0 + kchunk);
    zc acc = mk<double>(0, 0);
    for (int64_t k = k0 + threadIdx.x; k < k1; k += 256) cfmac(acc, a[k], b[k]);
    __shared__ zc red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)v * nchunk + c] = red[0];
}

__global__ __launch_bounds__(256) void k_dots_reduce(const zc* part, int nchunk, int nvec, zc* out) {
    const int v = (blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int lane = threadIdx.x % 64;
    if (v >= nvec) return;
    double re = 0.0, im = 0.0;
    for (int c = lane; c < nchunk; c += 64) {
        zc x = part[(size_t)v * nchunk + c];
        re += x.x;
        im += x.y;
    }
    for (int off = 32; off > 0; off >>= 1) {
        re += __shfl_down(re, off, 64);
        im += __shfl_down(im, off, 64);
    }
    if (lane == 0) out[v] = mk<double>(re, im);
}

// residual norms r_v = || h_v - theta_v s_v ||_2: one 1024-thread block per vector,
// four independent loads in flight per thread, wave shuffles then one LDS pass
__global__ __launch_bounds__(1024) void k_resid(const zc* const* th, const zc* const* ts, const double* theta,
                                                int64_t K, double* out) {
    const int v = blockIdx.x;
    const zc* h = th[v];
    const zc* s = ts[v];
    const double t = theta[v];
    double acc = 0.0;
    int64_t k = threadIdx.x;
    for (; k + 3 * 1024 < K; k += 4 * 1024) {
        zc a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] = h[k + u * 1024];
            b[u] = s[k + u * 1024];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double re = a[u].x - t * b[u].x, im = a[u].y - t * b[u].y;
            acc += re * re + im * im;
        }
    }
    for (; k < K; k += 1024) {
        const zc a = h[k], b = s[k];
        const double re = a.x - t * b.x, im = a.y - t * b.y;
        acc += re * re + im * im;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    __shared__ double red[16];
    if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int w = 0; w < 16; ++w) sum += red[w];
        out[v] = sqrt(sum);
    }
}

// Y_v[k] += sign * coef_v * X_v[k]
__global__ void k_axpy_tab(zc* const* ty, const zc* const* tx, const zc* coef, double sign, int64_t K) {
    const int v = blockIdx.y;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    zc c = cscale(coef[v], sign);
    zc* y = ty[v];
    cfma(y[k], c, tx[v][k]);
}

// X_v *= 1 / sqrt(re(d_v)) for every table entry (two tables scaled alike)
__global__ void k_normalize_tab(zc* const* t1, zc* const* t2, const zc* d, int64_t K) {
    const int v = blockIdx.y;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    // a vanished vector (converged seed) is zeroed; the projected problem deflates it
    double s = (d[v].x > 1e-280 && isfinite(d[v].x)) ? 1.0 / sqrt(d[v].x) : 0.0;
    t1[v][k] = cscale(t1[v][k], s);
    if (t2) t2[v][k] = cscale(t2[v][k], s);
}

// counter-based uniform numbers (splitmix64 of seed + index) in [-1, 1)
__device__ inline double u11(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ void k_random(zc* x, int nvec, int nb, int ld, int ng, uint64_t seed) {
    const int64_t K = (int64_t)nb * ld;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= K * nvec) return;
    int g = (int)(idx % ld);
    if (g >= ng) {
        x[idx] = mk<double>(0, 0);
        return;
    }
    uint64_t c = seed * 0x100000001B3ull + 2ull * (uint64_t)idx;
    x[idx] = mk<double>(u11(c), u11(c + 1));
}

// ---------------------------------------------------------------------------
// Batched generalized Hermitian eigenproblem H y = theta S y, N x N row-major.
// S = L L^H (right-looking Cholesky), A = L^{-1} H L^{-H}, cyclic Jacobi on A
// with the round-robin parallel ordering (N/2 disjoint rotations per step),
// Y = L^{-H} V, ascending order.  One workgroup per problem.
// ---------------------------------------------------------------------------
__device__ inline int rr_pair(int r, int k, int Np) {
    // circle method: players 0..Np-2 on the circle, Np-1 fixed
    return (r + k) % (Np - 1);
}

// largest projected problem (per-pair and per-root tables in LDS are sized by it)
constexpr int GENEIG_MAX = 512;

// Flags of the multi-workgroup Jacobi, after the nz problems' four N x N matrices:
// [0..2] any problem still rotating, one slot per sweep modulo 3; per problem z,
// [4 + 4z + 0..2] this problem still rotating (same slots) and [4 + 4z + 3] the copy
// of A (0 or 1) that holds its final matrix.
__device__ inline int* jacobi_flags(zc* gwork, int nz, size_t NN) {
    return reinterpret_cast<int*>(gwork + (size_t)nz * 4 * NN);
}

// the two rows of round r's pair pi (q = Np - 1 is the padding index when N is odd)
__device__ inline void rr_rows(int r, int pi, int Np, int& p, int& q) {
    if (pi == 0) { p = r % (Np - 1); q = Np - 1; }
    else { p = rr_pair(r, pi, Np); q = (r - pi + (Np - 1)) % (Np - 1); }
    if (p > q) { int t = p; p = q; q = t; }
}

// sweep limit of the projected eigen-solve
constexpr int GENEIG_SWEEPS = 60;

// squared relative size below which an off-diagonal element is not rotated
constexpr double JACOBI_TOL2 = 1e-28;

// MODE 2: the three work matrices (Cholesky factor L, A, V) live in LDS; MODE 1: A,
// which every Jacobi phase reads and writes, lives in LDS and L, V in global scratch
// (problems too large for all three); MODE 0: all in global scratch.  Pointers that
// derive from the shared array alone compile to LDS instructions (a pointer that may
// be either LDS or global memory would turn them into flat accesses).
// MODE 3 is the large-problem form: the matrices are in global scratch with room for
// a second copy of A, and the kernel runs in two parts around a Jacobi that spreads
// each round over many workgroups: PART 1 reduces to A (and V = I) and stops, PART 2
// orders and back-transforms from the copy of A the last sweep left (PART 0 is the
// whole solve in one workgroup).
template <int NT, int MODE, int PART = 0>
__global__ __launch_bounds__(NT) void k_geneig(const zc* Hs, const zc* Ss, int N, double* evals, zc* Ys,
                                               zc* gwork, int max_sweeps, int* status, int* sweeps_out) {
    extern __shared__ unsigned char sm[];
    const int z = blockIdx.x;
    const size_t NN = (size_t)N * N;
    const int NNi = N * N;  // 32-bit element index: no 64-bit division in the loops
    const zc* H = Hs + z * NN;
    const zc* S = Ss + z * NN;
    // three N x N work matrices: in LDS when they fit, else in global scratch
    zc* const G0 = gwork + z * (MODE == 3 ? 4 : 3) * NN;
    zc* Lg;  // Cholesky factor L
    zc* P1;  // work matrix, then A
    zc* P2;  // work matrix, then V
    if constexpr (MODE == 2) {
        Lg = reinterpret_cast<zc*>(sm);
        P1 = Lg + NN;
        P2 = Lg + 2 * NN;
    } else if constexpr (MODE == 1) {
        P1 = reinterpret_cast<zc*>(sm);
        Lg = G0;
        P2 = G0 + 2 * NN;
    } else {
        Lg = G0;
        P1 = G0 + NN;
        P2 = G0 + 2 * NN;
    }
    const int tid = threadIdx.x;
    __shared__ int bad;
    __shared__ int s_more;
    __shared__ int s_rot[2];
    __shared__ unsigned char dead[GENEIG_MAX];  // directions numerically in the span of earlier ones
    if (tid == 0) bad = 0;
    if constexpr (PART != 2) {
        // 1. Cholesky of S in P1; a pivot that lost all but 1e-8 of its diagonal marks a
        //    dependent direction: it is taken out of the reduction (unit pivot, zero column)
        //    and later pinned at the top of the spectrum so it is never selected
        for (int e = tid; e < NNi; e += NT) P1[e] = S[e];
        __syncthreads();
        for (int j = 0; j < N; ++j) {
            if (tid == 0) {
                double d = P1[(size_t)j * N + j].x;
                double d0 = S[(size_t)j * N + j].x;
                dead[j] = 0;
                if (!isfinite(d) || !isfinite(d0)) {
                    bad = 2;
                    d = 1.0;
                } else if (!(d > 1e-8 * d0) || !(d0 > 0.0)) {
                    dead[j] = 1;
                    d = 1.0;
                }
                P1[(size_t)j * N + j] = mk<double>(sqrt(d), 0.0);
            }
            __syncthreads();
            double inv = 1.0 / P1[(size_t)j * N + j].x;
            for (int i = j + 1 + tid; i < N; i += NT)
                P1[(size_t)i * N + j] = dead[j] ? mk<double>(0, 0) : cscale(P1[(size_t)i * N + j], inv);
            __syncthreads();
            // trailing update of the lower triangle: A_ik -= L_ij conj(L_kj), i >= k > j
            int w = N - j - 1;
            for (int e = tid; e < w * w; e += NT) {
                int i = j + 1 + e / w, k = j + 1 + e % w;
                if (k > i) continue;
                zc lij = P1[(size_t)i * N + j], lkj = P1[(size_t)k * N + j];
                zc t = mk<double>(lij.x * lkj.x + lij.y * lkj.y, lij.y * lkj.x - lij.x * lkj.y);  // lij conj(lkj)
                P1[(size_t)i * N + k] = csub(P1[(size_t)i * N + k], t);
            }
            __syncthreads();
        }
        for (int e = tid; e < NNi; e += NT) {
            int i = (int)(e / N), k = (int)(e % N);
            Lg[e] = (k <= i) ? P1[e] : mk<double>(0, 0);
        }
        // 2. B = L^{-1} H in P2 (column-wise forward substitution)
        for (int e = tid; e < NNi; e += NT) P2[e] = H[e];
        __syncthreads();
        for (int col = tid; col < N; col += NT) {
            for (int i = 0; i < N; ++i) {
                zc v = P2[(size_t)i * N + col];
    #pragma unroll 8
                for (int k = 0; k < i; ++k) v = csub(v, cmul(Lg[(size_t)i * N + k], P2[(size_t)k * N + col]));
                P2[(size_t)i * N + col] = cscale(v, 1.0 / Lg[(size_t)i * N + i].x);
            }
        }
        __syncthreads();
        // 3. A = L^{-1} B^H into P1: column j solves L a = conj(row j of B)
        for (int col = tid; col < N; col += NT) {
            for (int i = 0; i < N; ++i) {
                zc b = P2[(size_t)col * N + i];
                zc v = mk<double>(b.x, -b.y);
    #pragma unroll 8
                for (int k = 0; k < i; ++k) v = csub(v, cmul(Lg[(size_t)i * N + k], P1[(size_t)k * N + col]));
                P1[(size_t)i * N + col] = cscale(v, 1.0 / Lg[(size_t)i * N + i].x);
            }
        }
        __syncthreads();
        // 4. Hermitian part of A; V = I
        for (int e = tid; e < NNi; e += NT) {
            int i = (int)(e / N), k = (int)(e % N);
            if (k < i) {
                zc a = P1[(size_t)i * N + k], b = P1[(size_t)k * N + i];
                zc h = mk<double>(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
                P1[(size_t)i * N + k] = h;
                P1[(size_t)k * N + i] = mk<double>(h.x, -h.y);
            } else if (k == i) {
                P1[e] = mk<double>(P1[e].x, 0.0);
            }
            P2[e] = mk<double>(i == k ? 1.0 : 0.0, 0.0);
        }
        __syncthreads();
        for (int e = tid; e < NNi; e += NT) {
            int i = (int)(e / N), k = (int)(e % N);
            if (dead[i] || dead[k]) P1[e] = mk<double>(i == k ? 1e30 : 0.0, 0.0);
        }
        __syncthreads();
    }
    int* const jfl = jacobi_flags(gwork, gridDim.x, NN);
    if constexpr (PART == 1) {
        // the multi-workgroup sweeps start from A in the first copy; clear this
        // problem's per-sweep flags (and, once, the any-problem flags)
        if (tid == 0) {
            for (int k = 0; k < 4; ++k) jfl[4 + 4 * z + k] = 0;
            if (z == 0)
                for (int k = 0; k < 3; ++k) jfl[k] = 0;
            if (bad) atomicMax(status, bad);
        }
        return;
    }
    int sweep = 0;
    if constexpr (PART == 0) {
        // 5. cyclic Jacobi
        const int Np = N + (N & 1);
        const int npair = Np / 2;
        __shared__ double rc[GENEIG_MAX / 2], rsr[GENEIG_MAX / 2], rsi[GENEIG_MAX / 2];  // c, s e^{i phi} per pair
        __shared__ int rp[GENEIG_MAX / 2], rq[GENEIG_MAX / 2];
        for (; sweep < max_sweeps; ++sweep) {
            // converged when no off-diagonal element is above the rotation threshold
            // |a_pq| > 1e-14 (|a_pp| + |a_qq|): a smaller element changes the eigenvalues by
            // at most |a_pq|^2 / gap (or |a_pq| for a cluster), far below FP64 rounding of
            // the matrix itself, and rotating it only reshuffles rounding noise
            if (tid == 0) {
                s_more = 0;
                s_rot[0] = 0;
            }
            __syncthreads();
            int more = 0;
            for (int e = tid; e < NNi; e += NT) {
                const int i = e / N, k = e - i * N;
                if (k <= i || dead[i] || dead[k]) continue;  // deflated directions are already decoupled
                const zc a = P1[e];
                const double r2 = a.x * a.x + a.y * a.y;
                const double scale = fabs(P1[(size_t)i * N + i].x) + fabs(P1[(size_t)k * N + k].x);
                if (r2 > 1e-300 && r2 > JACOBI_TOL2 * scale * scale) more = 1;
            }
            if (more) s_more = 1;
            __syncthreads();
            if (!s_more) break;
            for (int r = 0; r < Np - 1; ++r) {
                // rotation of every pair of this round from its pivots a_pp, a_qq, a_pq
                // (the pairs are disjoint, so no pair's pivots change within the round).
                // s_rot[r & 1] records whether any pair rotates; the flag of the next round
                // is cleared here, before this round's barrier, so it is clear before any
                // thread can set it
                if (tid == 0) s_rot[(r + 1) & 1] = 0;
                for (int pi = tid; pi < npair; pi += NT) {
                    int p, q;
                    if (pi == 0) { p = r % (Np - 1); q = Np - 1; }
                    else { p = rr_pair(r, pi, Np); q = (r - pi + (Np - 1)) % (Np - 1); }
                    if (p > q) { int t = p; p = q; q = t; }
                    double c = 1.0, sr = 0.0, si = 0.0;
                    if (q < N) {
                        const zc apq = P1[(size_t)p * N + q];
                        const double r2 = apq.x * apq.x + apq.y * apq.y;
                        const double app = P1[(size_t)p * N + p].x, aqq = P1[(size_t)q * N + q].x;
                        const double scale = fabs(app) + fabs(aqq);
                        if (r2 > 1e-300 && r2 > JACOBI_TOL2 * scale * scale) {
                            // tan of the rotation angle: t = 2|a_pq| sgn(d) / (|d| + sqrt(d^2 + 4|a_pq|^2)),
                            // d = a_qq - a_pp; c = 1/sqrt(1 + t^2); phase a_pq / |a_pq|
                            const double d = aqq - app;
                            const double inv_r = rsqrt(r2);
                            const double rabs = r2 * inv_r;
                            const double t = (d >= 0 ? 2.0 : -2.0) * rabs / (fabs(d) + sqrt(d * d + 4.0 * r2));
                            c = rsqrt(1.0 + t * t);
                            const double sn = t * c * inv_r;
                            sr = sn * apq.x;  // s e^{i phi}
                            si = sn * apq.y;
                        }
                    }
                    rc[pi] = c; rsr[pi] = sr; rsi[pi] = si; rp[pi] = p; rq[pi] = q;
                    if (sr != 0.0 || si != 0.0) s_rot[r & 1] = 1;
                }
                __syncthreads();
                if (!s_rot[r & 1]) continue;  // nothing rotates this round (uniform branch)
                // One pass over A and V.  A: every 2x2 block (rows of pair ia, columns of
                // pair ib) is owned by one thread, which applies the row rotation of pair ia
                //   a_pj' = c a_pj - s e^{i phi} a_qj ; a_qj' = s e^{-i phi} a_pj + c a_qj
                // and then the column rotation of pair ib
                //   a_ip' = c a_ip - s e^{-i phi} a_iq ; a_iq' = s e^{i phi} a_ip + c a_iq
                // (the pairs are disjoint, so this equals a full row pass followed by a full
                // column pass, operation for operation).  V: columns p, q of every pair.
                {
                    const int nblk = npair * npair;
                    for (int e = tid; e < nblk + npair * N; e += NT) {
                        if (e < nblk) {
                            const int ia = e / npair, ib = e - ia * npair;
                            const int pa = rp[ia], qa = rq[ia], pb = rp[ib], qb = rq[ib];
                            const bool va = qa < N, vb = qb < N;  // second row / column exists
                            const bool ra = va && (rsr[ia] != 0.0 || rsi[ia] != 0.0);
                            const bool rb = vb && (rsr[ib] != 0.0 || rsi[ib] != 0.0);
                            if (!ra && !rb) continue;
                            const zc zero = mk<double>(0, 0);
                            zc x00 = P1[(size_t)pa * N + pb];
                            zc x01 = vb ? P1[(size_t)pa * N + qb] : zero;
                            zc x10 = va ? P1[(size_t)qa * N + pb] : zero;
                            zc x11 = (va && vb) ? P1[(size_t)qa * N + qb] : zero;
                            if (ra) {
                                const double c = rc[ia];
                                const zc se = mk<double>(rsr[ia], rsi[ia]);
                                const zc sec = mk<double>(rsr[ia], -rsi[ia]);
                                const zc n00 = csub(cscale(x00, c), cmul(se, x10));
                                const zc n10 = cadd(cmul(sec, x00), cscale(x10, c));
                                x00 = n00;
                                x10 = n10;
                                if (vb) {
                                    const zc n01 = csub(cscale(x01, c), cmul(se, x11));
                                    const zc n11 = cadd(cmul(sec, x01), cscale(x11, c));
                                    x01 = n01;
                                    x11 = n11;
                                }
                            }
                            if (rb) {
                                const double c = rc[ib];
                                const zc se = mk<double>(rsr[ib], rsi[ib]);
                                const zc sec = mk<double>(rsr[ib], -rsi[ib]);
                                const zc n00 = csub(cscale(x00, c), cmul(sec, x01));
                                const zc n01 = cadd(cmul(se, x00), cscale(x01, c));
                                x00 = n00;
                                x01 = n01;
                                if (va) {
                                    const zc n10 = csub(cscale(x10, c), cmul(sec, x11));
                                    const zc n11 = cadd(cmul(se, x10), cscale(x11, c));
                                    x10 = n10;
                                    x11 = n11;
                                }
                            }
                            P1[(size_t)pa * N + pb] = x00;
                            if (vb) P1[(size_t)pa * N + qb] = x01;
                            if (va) P1[(size_t)qa * N + pb] = x10;
                            if (va && vb) P1[(size_t)qa * N + qb] = x11;
                        } else {
                            const int f = e - nblk;
                            const int pi = f / N, i = f - pi * N;
                            const int p = rp[pi], q = rq[pi];
                            if (q >= N || (rsr[pi] == 0.0 && rsi[pi] == 0.0)) continue;
                            const double c = rc[pi];
                            const zc se = mk<double>(rsr[pi], rsi[pi]);
                            const zc sec = mk<double>(rsr[pi], -rsi[pi]);
                            const zc vp = P2[(size_t)i * N + p], vq = P2[(size_t)i * N + q];
                            P2[(size_t)i * N + p] = csub(cscale(vp, c), cmul(sec, vq));
                            P2[(size_t)i * N + q] = cadd(cmul(se, vp), cscale(vq, c));
                        }
                    }
                }
                __syncthreads();
            }
        }
    }
    if constexpr (PART == 2) P1 = G0 + NN + (size_t)jfl[4 + 4 * z + 3] * 2 * NN;  // copy of A the sweeps ended in
    // 6. order and back-transform in LDS: Yl = L^{-H} V (into P1 once the eigenvalues
    //    are saved), then column j of Yl goes to column rank(j) of Y
    __shared__ double evs[GENEIG_MAX];
    __shared__ int rk[GENEIG_MAX];
    for (int j = tid; j < N; j += NT) evs[j] = P1[(size_t)j * N + j].x;
    __syncthreads();
    for (int j = tid; j < N; j += NT) {
        const double dj = evs[j];
        int rank = 0;
        for (int i = 0; i < N; ++i) {
            const double di = evs[i];
            if (di < dj || (di == dj && i < j)) ++rank;
        }
        rk[j] = rank;
        if (!isfinite(dj)) bad = 2;
        // L^H y = v, back substitution down the column
        for (int i = N - 1; i >= 0; --i) {
            zc v = P2[(size_t)i * N + j];
#pragma unroll 8
            for (int k = i + 1; k < N; ++k) {
                const zc l = Lg[(size_t)k * N + i];
                const zc yk = P1[(size_t)k * N + j];
                v = csub(v, mk<double>(l.x * yk.x + l.y * yk.y, l.x * yk.y - l.y * yk.x));  // conj(l) yk
            }
            P1[(size_t)i * N + j] = cscale(v, 1.0 / Lg[(size_t)i * N + i].x);
        }
    }
    __syncthreads();
    double* ev = evals + (size_t)z * N;
    zc* Y = Ys + z * NN;
    for (int j = tid; j < N; j += NT) ev[rk[j]] = evs[j];
    for (int e = tid; e < NNi; e += NT) {
        const int i = (int)(e / N), j = (int)(e % N);
        Y[(size_t)i * N + rk[j]] = P1[e];
    }
    if (tid == 0 && bad) atomicMax(status, bad);
    if constexpr (PART == 0)
        if (tid == 0 && sweeps_out) sweeps_out[z] = sweep;
}

// ---------------------------------------------------------------------------
// Multi-workgroup cyclic Jacobi on A (the large-problem form, between the two parts
// of k_geneig<.., 3, ..>).  The same rotations as the one-workgroup sweep, in the same
// round-robin order, but one launch per round: block pi of a round owns rows p, q of
// its pair.  Every block derives all the round's rotations from the pivots of the
// round's input copy of A, applies its own rotation to rows p, q and every pair's
// rotation to the columns, and writes rows p, q of the other copy; V = V J is applied
// to rows p, q of V in place.  Copies alternate every round, so sweep s starts from
// copy s & 1 (a sweep has an odd number of rounds).
// ---------------------------------------------------------------------------
// sweep s's check: is any off-diagonal element above the rotation threshold?
__global__ __launch_bounds__(256) void k_jacobi_check(zc* gwork, int N, int s, int* sweeps_out) {
    const int z = blockIdx.y, nz = gridDim.y;
    const size_t NN = (size_t)N * N;
    int* const fl = jacobi_flags(gwork, nz, NN);
    int* const mine = fl + 4 + 4 * z;
    const int cur = s % 3, prev = (s + 2) % 3, next = (s + 1) % 3;
    if (s > 0 && mine[prev] == 0) return;  // converged at an earlier check
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        mine[next] = 0;
        mine[3] = s & 1;
        if (sweeps_out) sweeps_out[z] = s;
        if (z == 0) fl[next] = 0;
    }
    const zc* A = gwork + (size_t)z * 4 * NN + NN + (size_t)(s & 1) * 2 * NN;
    const int NNi = N * N;
    int more = 0;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < NNi; e += gridDim.x * 256) {
        const int i = e / N, k = e - i * N;
        if (k <= i) continue;
        const zc a = A[e];
        const double r2 = a.x * a.x + a.y * a.y;
        const double scale = fabs(A[(size_t)i * N + i].x) + fabs(A[(size_t)k * N + k].x);
        if (r2 > 1e-300 && r2 > JACOBI_TOL2 * scale * scale) more = 1;
    }
    if (__syncthreads_or(more) && threadIdx.x == 0) {
        atomicOr(&mine[cur], 1);
        atomicOr(&fl[cur], 1);
    }
}

// round r of sweep s; grid (N_p / 2 pairs, problems), 256 threads
__global__ __launch_bounds__(256) void k_jacobi_round(zc* gwork, int N, int s, int r) {
    const int z = blockIdx.y, nz = gridDim.y;
    const size_t NN = (size_t)N * N;
    if (jacobi_flags(gwork, nz, NN)[4 + 4 * z + s % 3] == 0) return;  // converged
    const int Np = N + (N & 1), npair = Np / 2;
    const int in = (int)(((long long)s * (Np - 1) + r) & 1);
    zc* const G0 = gwork + (size_t)z * 4 * NN;
    const zc* const A = G0 + NN + (size_t)in * 2 * NN;
    zc* const Ao = G0 + NN + (size_t)(in ^ 1) * 2 * NN;
    zc* const V = G0 + 2 * NN;
    __shared__ double rc[GENEIG_MAX / 2], rsr[GENEIG_MAX / 2], rsi[GENEIG_MAX / 2];
    __shared__ int rp[GENEIG_MAX / 2], rq[GENEIG_MAX / 2];
    const int tid = threadIdx.x;
    for (int pi = tid; pi < npair; pi += 256) {
        int p, q;
        rr_rows(r, pi, Np, p, q);
        double c = 1.0, sr = 0.0, si = 0.0;
        if (q < N) {
            const zc apq = A[(size_t)p * N + q];
            const double r2 = apq.x * apq.x + apq.y * apq.y;
            const double app = A[(size_t)p * N + p].x, aqq = A[(size_t)q * N + q].x;
            const double scale = fabs(app) + fabs(aqq);
            if (r2 > 1e-300 && r2 > JACOBI_TOL2 * scale * scale) {
                // same rotation as the one-workgroup sweep: tan t from d = a_qq - a_pp
                const double d = aqq - app;
                const double inv_r = rsqrt(r2);
                const double rabs = r2 * inv_r;
                const double tn = (d >= 0 ? 2.0 : -2.0) * rabs / (fabs(d) + sqrt(d * d + 4.0 * r2));
                c = rsqrt(1.0 + tn * tn);
                const double sn = tn * c * inv_r;
                sr = sn * apq.x;
                si = sn * apq.y;
            }
        }
        rc[pi] = c; rsr[pi] = sr; rsi[pi] = si; rp[pi] = p; rq[pi] = q;
    }
    __syncthreads();
    const int me = blockIdx.x;
    const int p0 = rp[me], q0 = rq[me];
    const bool hq0 = q0 < N;
    const double c0 = rc[me];
    const zc se0 = mk<double>(rsr[me], rsi[me]), sec0 = mk<double>(rsr[me], -rsi[me]);
    const zc zero = mk<double>(0.0, 0.0);
    for (int cp = tid; cp < npair; cp += 256) {
        const int p1 = rp[cp], q1 = rq[cp];
        const bool hq1 = q1 < N;
        const double c1 = rc[cp];
        const zc se1 = mk<double>(rsr[cp], rsi[cp]), sec1 = mk<double>(rsr[cp], -rsi[cp]);
        // the 2 x 2 block of A at rows (p0, q0), columns (p1, q1): rows first
        // (x_p' = c x_p - s e^{i phi} x_q, x_q' = s e^{-i phi} x_p + c x_q), then columns
        // (y_p' = c y_p - s e^{-i phi} y_q, y_q' = s e^{i phi} y_p + c y_q)
        const zc a00 = A[(size_t)p0 * N + p1];
        const zc a01 = hq1 ? A[(size_t)p0 * N + q1] : zero;
        const zc a10 = hq0 ? A[(size_t)q0 * N + p1] : zero;
        const zc a11 = hq0 && hq1 ? A[(size_t)q0 * N + q1] : zero;
        const zc b00 = csub(cscale(a00, c0), cmul(se0, a10)), b10 = cadd(cmul(sec0, a00), cscale(a10, c0));
        const zc b01 = csub(cscale(a01, c0), cmul(se0, a11)), b11 = cadd(cmul(sec0, a01), cscale(a11, c0));
        Ao[(size_t)p0 * N + p1] = csub(cscale(b00, c1), cmul(sec1, b01));
        if (hq1) Ao[(size_t)p0 * N + q1] = cadd(cmul(se1, b00), cscale(b01, c1));
        if (hq0) {
            Ao[(size_t)q0 * N + p1] = csub(cscale(b10, c1), cmul(sec1, b11));
            if (hq1) Ao[(size_t)q0 * N + q1] = cadd(cmul(se1, b10), cscale(b11, c1));
        }
        // rows p0, q0 of V at columns (p1, q1), column rotation only (skipped when
        // the pair does not rotate, as in the one-workgroup sweep)
        if (hq1 && (rsr[cp] != 0.0 || rsi[cp] != 0.0)) {
            const int rows[2] = {p0, q0};
            for (int k = 0; k < (hq0 ? 2 : 1); ++k) {
                const size_t o = (size_t)rows[k] * N;
                const zc vp = V[o + p1], vq = V[o + q1];
                V[o + p1] = csub(cscale(vp, c1), cmul(sec1, vq));
                V[o + q1] = cadd(cmul(se1, vp), cscale(vq, c1));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Block selection: per block z with nr = b + m Ritz pairs (ascending) and the
// b inputs as its first basis vectors, pick for each input slot the Ritz vector
// of largest |<y_r|S|x_a>|^2 = |Y[a][r]|^2 (greedy, largest overlaps first);
// then any unpicked Ritz value among the b lowest replaces the highest picked
// one (new roots).  Writes coefficient columns C_z (nr x b) and theta.
// ---------------------------------------------------------------------------
// map (optional): block z's roots go to theta_out[map[z] * b + a] (a subset of the blocks)
__global__ void k_select(const zc* Ys, const double* ev, int nr, int b, zc* C, double* theta_out, int nblocks,
                         const int32_t* map) {
    const int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= nblocks) return;
    const zc* Y = Ys + (size_t)z * nr * nr;
    const double* e = ev + (size_t)z * nr;
    int pick[32];
    bool used[64];
    bool done[32];
    for (int r = 0; r < nr; ++r) used[r] = false;
    for (int a = 0; a < b; ++a) { pick[a] = -1; done[a] = false; }
    for (int it = 0; it < b; ++it) {
        double best = -1.0;
        int ba = 0, br = 0;
        for (int a = 0; a < b; ++a) {
            if (done[a]) continue;
            for (int r = 0; r < nr; ++r) {
                if (used[r]) continue;
                zc y = Y[(size_t)a * nr + r];
                double o = y.x * y.x + y.y * y.y;
                if (o > best) { best = o; ba = a; br = r; }
            }
        }
        pick[ba] = br;
        done[ba] = true;
        used[br] = true;
    }
    for (int r = 0; r < b; ++r) {
        if (used[r]) continue;
        int worst = 0;
        for (int a = 1; a < b; ++a)
            if (pick[a] > pick[worst]) worst = a;
        if (pick[worst] > r) {
            used[pick[worst]] = false;
            pick[worst] = r;
            used[r] = true;
        }
    }
    for (int a = 0; a < b; ++a) {
        int r = pick[a];
        theta_out[(size_t)(map ? map[z] : z) * b + a] = e[r];
        for (int i = 0; i < nr; ++i) C[((size_t)z * nr + i) * b + a] = Y[(size_t)i * nr + r];
    }
}

// dst[v][k] = src[v][k] for v < n (blockIdx.y), k < K
__global__ void k_copy_tab(zc* const* dst, const zc* const* src, int64_t K) {
    const zc* a = src[blockIdx.y];
    zc* o = dst[blockIdx.y];
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < K; k += (int64_t)gridDim.x * blockDim.x)
        o[k] = a[k];
}

__global__ void k_copy_cols(const zc* Y, int ldy, int ncols, int nrows, zc* out) {
    // out (nrows x ncols, row-major) = first ncols columns of Y (nrows x ldy)
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nrows * ncols) return;
    int i = e / ncols, j = e % ncols;
    out[e] = Y[(size_t)i * ldy + j];
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static bool gram64_enabled() {
    static const bool on = [] {
        const char* e = getenv("MBKS_GRAM64");
        return !(e && e[0] == '0');
    }();
    return on;
}

// the wide Gram products run on the FP64 matrix cores unless MBKS_GRAM_MFMA=0 (read per
// call, for cross-checks against the vector kernel)
static bool gram_mfma_enabled() {
    const char* e = getenv("MBKS_GRAM_MFMA");
    return !(e && e[0] == '0');
}

// MBKS_GRAM_HERM=0 computes Hermitian products on every tile (for cross-checks)
static bool gram_herm_enabled() {
    const char* e = getenv("MBKS_GRAM_HERM");
    return !(e && e[0] == '0');
}

mb_status dense_gram(const void* const* ta, const void* const* tb, int MA, int NB, int nz, int64_t K, void* out,
                     void* scratch, size_t scratch_bytes, hipStream_t s, bool herm) {
    if (MA <= 0 || NB <= 0 || nz <= 0) return MB_OK;
    const bool tiny = MA <= TINY && NB <= TINY;  // all outputs of a chunk in one block
    const bool skinny = !tiny && MA <= SKINNY;    // one block per output column
    const bool big = !tiny && !skinny && MA > GT && NB > GT;  // 32 x 32 tiles for the wide products
    // 64 x 64 tiles from 256 up (measured: 1.3x faster than 32 x 32 tiles at
    // MA, NB ~ 340-1000, slower at ~ 100-250, where the grid has too few blocks)
    const bool wide = big && MA >= 256 && NB >= 256 && gram64_enabled();
    const int tile = wide ? G64 : big ? GT2 : GT, kstep = (tiny || skinny) ? 256 : wide ? GK64 : big ? GK2 : GK;
    int tiles_m = (MA + tile - 1) / tile, tiles_n = (NB + tile - 1) / tile;
    // Hermitian products on the matrix cores: the upper tiles only
    const bool htri = herm && MA == NB && wide && gram_mfma_enabled() && gram_herm_enabled();
    int ntiles = tiny ? nz : skinny ? NB * nz : (htri ? tiles_m * (tiles_m + 1) / 2 : tiles_m * tiles_n) * nz;
    // at least 256 (64 for the wide tiles) k per chunk; about 1024 blocks in all
    // (4096 for the narrow kernel, whose blocks are short; the tiny kernel's blocks end
    // in a reduction of up to 64 sums, so they take longer k ranges)
    int64_t maxchunk = big ? (K + 63) / 64 : (K + 255) / 256;
    const int target = skinny ? 4096 : tiny ? 512 : 1024;
    int nchunk = (int)std::max<int64_t>(1, std::min<int64_t>(maxchunk, target / std::max(1, ntiles)));
    size_t need = (size_t)nz * nchunk * MA * NB * sizeof(zc);
    while (need > scratch_bytes && nchunk > 1) {
        nchunk /= 2;
        need = (size_t)nz * nchunk * MA * NB * sizeof(zc);
    }
    if (need > scratch_bytes) return set_error(MB_ERR_INVALID_ARG, "gram scratch too small");
    int64_t kchunk = (K + nchunk - 1) / nchunk;
    kchunk = (kchunk + kstep - 1) / kstep * kstep;
    nchunk = (int)((K + kchunk - 1) / kchunk);
    dim3 grid(nchunk, tiny ? 1 : skinny ? NB : tiles_m * tiles_n, nz);
    StageScope ts_(MB_STAGE_GRAM, s);
    if (tiny)
        hipLaunchKernelGGL(k_gram_tiny, grid, dim3(256), 0, s, (const zc* const*)ta, (const zc* const*)tb, MA, NB,
                           K, kchunk, nchunk, (zc*)scratch);
    else if (skinny)
        hipLaunchKernelGGL(k_gram_skinny, grid, dim3(256), 0, s, (const zc* const*)ta, (const zc* const*)tb, MA, NB,
                           K, kchunk, nchunk, (zc*)scratch);
    else if (wide && gram_mfma_enabled())
        hipLaunchKernelGGL(k_gram_mfma,
                           dim3((unsigned)((htri ? tiles_m * (tiles_m + 1) / 2 : tiles_m * tiles_n) * nchunk * nz)),
                           dim3(256), 0, s, (const zc* const*)ta, (const zc* const*)tb, MA, NB, K, kchunk, nchunk,
                           tiles_m, tiles_n, (zc*)scratch, htri ? 1 : 0);
    else if (wide)
        hipLaunchKernelGGL(k_gram64, dim3((unsigned)(tiles_m * tiles_n * nchunk * nz)), dim3(256), 0, s,
                           (const zc* const*)ta, (const zc* const*)tb, MA, NB, K, kchunk, nchunk, tiles_m, tiles_n,
                           (zc*)scratch);
    else if (big)
        hipLaunchKernelGGL(k_gram32, grid, dim3(256), 0, s, (const zc* const*)ta, (const zc* const*)tb, MA, NB, K,
                           kchunk, nchunk, tiles_n, (zc*)scratch);
    else
        hipLaunchKernelGGL(k_gram, grid, dim3(256), 0, s, (const zc* const*)ta, (const zc* const*)tb, MA, NB, K,
                           kchunk, nchunk, tiles_n, (zc*)scratch);
    MB_HIP_TRY(hipGetLastError());
    size_t tot = (size_t)MA * NB * nz;
    hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((tot * 64 + 255) / 256)), dim3(256), 0, s, (const zc*)scratch,
                       (zc*)out, MA, NB, nchunk, nz, htri ? tile : 0);
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

mb_status dense_combo(const void* const* tx, void* const* ty, const void* W, int MI, int NO, int nz, int64_t K,
                      double alpha, double beta, hipStream_t s, bool low) {
    if (MI <= 0 || NO <= 0 || nz <= 0) return MB_OK;
    StageScope ts_(MB_STAGE_COMBO, s);
    static const int cw_env = [] {
        const char* e = getenv("MBKS_COMBO_CW");
        return e ? atoi(e) : -1;
    }();
    // 16 outputs per thread for the wide combinations (measured 1.8x faster than 8 on
    // MI, NO ~ 300-1000), 8 for the narrow ones, whose grids would otherwise be small
    const int cw = (cw_env == 8 || cw_env == 16 || cw_env == 32) ? cw_env : (MI >= 64 && NO >= 64) ? 16 : 8;
    // wide combinations (both sides >= 128, e.g. the rotations and Gram-Schmidt updates of
    // hundreds of trial vectors) on the matrix cores; MBKS_COMBO_MFMA=0 keeps them on the
    // vector units (cross-checks)
    const char* me = getenv("MBKS_COMBO_MFMA");
    const bool mfma_on = !(me && me[0] == '0');
    if (mfma_on && cw_env < 0 && MI >= 128 && NO >= 128 && K >= 4096) {
        const int nng = (NO + CM_N - 1) / CM_N;
        const int64_t nkb = (K + CM_K - 1) / CM_K;
        if ((int64_t)nng * nkb < ((int64_t)1 << 31)) {
            if (low)
                hipLaunchKernelGGL(k_combo_mfma32, dim3((unsigned)(nng * nkb), nz), dim3(256), 0, s,
                                   (const zc* const*)tx, (zc* const*)ty, (const zc*)W, MI, NO, K, alpha, beta, nng, nkb);
            else
                hipLaunchKernelGGL(k_combo_mfma, dim3((unsigned)(nng * nkb), nz), dim3(256), 0, s,
                                   (const zc* const*)tx, (zc* const*)ty, (const zc*)W, MI, NO, K, alpha, beta, nng, nkb);
            MB_HIP_TRY(hipGetLastError());
            return MB_OK;
        }
    }
    if (cw == 8) launch_combo_w<8>(tx, ty, W, MI, NO, nz, K, alpha, beta, s);
    else if (cw == 16) launch_combo_w<16>(tx, ty, W, MI, NO, nz, K, alpha, beta, s);
    else launch_combo_w<32>(tx, ty, W, MI, NO, nz, K, alpha, beta, s);
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

mb_status dense_dots(const void* const* ta, const void* const* tb, int nvec, int64_t K, void* out, void* scratch,
                     hipStream_t s) {
    StageScope ts_(MB_STAGE_OTHER, s);
    if (nvec <= 0) return MB_OK;
    // about 1024 blocks in total, at least 4096 elements per block
    int nchunk = (int)std::max<int64_t>(1, std::min<int64_t>((K + 4095) / 4096, 1024 / nvec));
    nchunk = std::min(nchunk, 64);
    int64_t kchunk = (K + nchunk - 1) / nchunk;
    hipLaunchKernelGGL(k_dots, dim3(nchunk, nvec), dim3(256), 0, s, (const zc* const*)ta, (const zc* const*)tb, K,
                       kchunk, nchunk, (zc*)scratch);
    MB_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_dots_reduce, dim3((nvec * 64 + 255) / 256), dim3(256), 0, s, (const zc*)scratch, nchunk,
                       nvec, (zc*)out);
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

mb_status dense_resid(const void* const* th, const void* const* ts, const double* theta, int nvec, int64_t K,
                      double* out, hipStream_t s) {
    StageScope ts_(MB_STAGE_OTHER, s);
    if (nvec <= 0) return MB_OK;
    hipLaunchKernelGGL(k_resid, dim3(nvec), dim3(1024), 0, s, (const zc* const*)th, (const zc* const*)ts, theta, K,
                       out);
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

mb_status dense_axpy(void* const* ty, const void* const* tx, const void* coef, double sign, int nvec, int64_t K,
                     hipStream_t s) {
    StageScope ts_(MB_STAGE_OTHER, s);
    if (nvec <= 0) return MB_OK;
    dim3 grid((unsigned)((K + 255) / 256), nvec);
    hipLaunchKernelGGL(k_axpy_tab, grid, dim3(256), 0, s, (zc* const*)ty, (const zc* const*)tx, (const zc*)coef, sign,
                       K);
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

mb_status dense_normalize(void* const* t1, void* const* t2, const void* d, int nvec, int64_t K, hipStream_t s) {
    StageScope ts_(MB_STAGE_OTHER, s);
    if (nvec <= 0) return MB_OK;
    dim3 grid((unsigned)((K + 255) / 256), nvec);
    hipLaunchKernelGGL(k_normalize_tab, grid, dim3(256), 0, s, (zc* const*)t1, (zc* const*)t2, (const zc*)d, K);
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

mb_status dense_random(void* x, int nvec, int nb, int ld, int ng, uint64_t seed, hipStream_t s) {
    StageScope ts_(MB_STAGE_OTHER, s);
    int64_t tot = (int64_t)nvec * nb * ld;
    hipLaunchKernelGGL(k_random, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, (zc*)x, nvec, nb, ld, ng, seed);
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

mb_status dense_geneig(const void* H, const void* S, int N, int nz, double* evals, void* Y, void* gwork,
                       int* status, hipStream_t s, int* sweeps) {
    if (N <= 0 || nz <= 0) return MB_OK;
    if (N > GENEIG_MAX) return set_error(MB_ERR_INVALID_ARG, "projected problem larger than 512");
    const size_t nn16 = (size_t)N * N * sizeof(zc);
    const int mode = 3 * nn16 <= 150000 ? 2 : nn16 <= 150000 ? 1 : 0;
    const size_t dyn = mode == 2 ? 3 * nn16 : mode == 1 ? nn16 : 0;
    StageScope ts_(MB_STAGE_SMALLEIG, s);
    // one wave for the smallest problems; otherwise 1024 threads (measured on N = 16-34:
    // 1.0-1.5x faster than 256 threads, 1.3-2.7x faster than 64)
    const int nt = N <= 12 ? 64 : 1024;
    auto launch = [&](auto kern, int threads) -> mb_status {
        if (dyn > 65536)
            MB_HIP_TRY(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
        hipLaunchKernelGGL(kern, dim3(nz), dim3(threads), dyn, s, (const zc*)H, (const zc*)S, N, evals, (zc*)Y,
                           (zc*)gwork, GENEIG_SWEEPS, status, sweeps);
        return MB_OK;
    };
    mb_status st;
    if (mode == 0) {
        // large problems: reduction and back-transform in one workgroup per problem,
        // the Jacobi sweeps spread over N/2 workgroups per problem, one launch per
        // round; the host reads the any-problem flag after each sweep's check
        st = launch(k_geneig<1024, 3, 1>, 1024);
        if (st != MB_OK) return st;
        const int Np = N + (N & 1);
        const int nchk = (int)std::min<size_t>(64, ((size_t)N * N + 2047) / 2048);
        const int* any = reinterpret_cast<const int*>((const zc*)gwork + (size_t)nz * 4 * N * N);
        for (int sw = 0;; ++sw) {
            hipLaunchKernelGGL(k_jacobi_check, dim3(nchk, nz), dim3(256), 0, s, (zc*)gwork, N, sw, sweeps);
            MB_HIP_TRY(hipGetLastError());
            int more = 0;
            MB_HIP_TRY(hipMemcpyAsync(&more, any + sw % 3, sizeof(int), hipMemcpyDeviceToHost, s));
            MB_HIP_TRY(hipStreamSynchronize(s));
            if (!more || sw == GENEIG_SWEEPS) break;
            for (int r = 0; r < Np - 1; ++r)
                hipLaunchKernelGGL(k_jacobi_round, dim3(Np / 2, nz), dim3(256), 0, s, (zc*)gwork, N, sw, r);
            MB_HIP_TRY(hipGetLastError());
        }
        st = launch(k_geneig<1024, 3, 2>, 1024);
    } else if (mode == 1)
        st = launch(k_geneig<1024, 1>, 1024);
    else if (nt == 64)
        st = launch(k_geneig<64, 2>, 64);
    else
        st = launch(k_geneig<1024, 2>, 1024);
    if (st != MB_OK) return st;
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

size_t geneig_work_bytes(int N, int nz) {
    return (size_t)4 * N * N * nz * sizeof(zc) + 16 * (size_t)nz + 64;
}

mb_status dense_select(const void* Y, const double* ev, int nr, int b, void* C, double* theta, int nblocks,
                       hipStream_t s, const int32_t* map) {
    StageScope ts_(MB_STAGE_OTHER, s);
    if (b > 32 || nr > 64) return set_error(MB_ERR_INVALID_ARG, "block too large for selection");
    hipLaunchKernelGGL(k_select, dim3((nblocks + 63) / 64), dim3(64), 0, s, (const zc*)Y, ev, nr, b, (zc*)C, theta,
                       nblocks, map);
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

mb_status dense_copy_tab(void* const* dst, const void* const* src, int n, int64_t K, hipStream_t s) {
    if (n <= 0 || K <= 0) return MB_OK;
    if (n > 65535) return set_error(MB_ERR_INVALID_ARG, "dense_copy_tab: too many vectors");
    StageScope ts_(MB_STAGE_OTHER, s);
    const unsigned gx = (unsigned)std::min<int64_t>((K + 255) / 256, 256);
    hipLaunchKernelGGL(k_copy_tab, dim3(gx, (unsigned)n), dim3(256), 0, s, (zc* const*)dst, (const zc* const*)src, K);
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

mb_status dense_copy_cols(const void* Y, int ldy, int ncols, int nrows, void* out, hipStream_t s) {
    StageScope ts_(MB_STAGE_OTHER, s);
    int tot = nrows * ncols;
    hipLaunchKernelGGL(k_copy_cols, dim3((tot + 255) / 256), dim3(256), 0, s, (const zc*)Y, ldy, ncols, nrows,
                       (zc*)out);
    MB_HIP_TRY(hipGetLastError());
    return MB_OK;
}

}  // namespace mb

extern "C" mb_status mb_small_geneig(const double* H, const double* S, int N, int nz, double* evals, double* Y,
                                     int* sweeps, void* stream) {
    using namespace mb;
    if (!H || !S || !evals || !Y || N < 1 || N > GENEIG_MAX || nz < 1 || nz > 4096)
        return set_error(MB_ERR_INVALID_ARG, "mb_small_geneig: bad arguments");
    hipStream_t s = (hipStream_t)stream;
    const size_t nn = (size_t)N * N * nz;
    void *dH = nullptr, *dS = nullptr, *dY = nullptr, *dW = nullptr;
    double* dE = nullptr;
    int *dst = nullptr, *dsw = nullptr;
    auto cleanup = [&]() {
        (void)hipFree(dH); (void)hipFree(dS); (void)hipFree(dY); (void)hipFree(dW);
        (void)hipFree(dE); (void)hipFree(dst); (void)hipFree(dsw);
    };
    {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
            (void)hipGetLastError();
            return set_error(MB_ERR_NO_DEVICE, "mb_small_geneig: no GPU");
        }
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;
        (void)hipSetDevice(dev);
        (void)hipGetLastError();
    }
    void** bufs[] = {&dH, &dS, &dY, &dW, (void**)&dE, (void**)&dst, (void**)&dsw};
    const size_t sizes[] = {nn * 16, nn * 16, nn * 16, geneig_work_bytes(N, nz), (size_t)N * nz * 8, 64, (size_t)nz * 4 + 64};
    for (int k = 0; k < 7; ++k) {
        hipError_t e = hipMalloc(bufs[k], sizes[k]);
        if (e != hipSuccess) {
            cleanup();
            return set_error(MB_ERR_OOM, std::string("mb_small_geneig: hipMalloc: ") + hipGetErrorString(e));
        }
    }
    mb_status st = MB_OK;
    int status = 0;
    if (hipMemcpy(dH, H, nn * 16, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dS, S, nn * 16, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(dst, 0, 4) != hipSuccess) {
        cleanup();
        return set_error(MB_ERR_HIP, "mb_small_geneig: upload failed");
    }
    st = dense_geneig(dH, dS, N, nz, dE, dY, dW, dst, s, dsw);
    if (st == MB_OK) {
        if (hipStreamSynchronize(s) != hipSuccess ||
            hipMemcpy(evals, dE, (size_t)N * nz * 8, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(Y, dY, nn * 16, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(&status, dst, 4, hipMemcpyDeviceToHost) != hipSuccess ||
            (sweeps && hipMemcpy(sweeps, dsw, (size_t)nz * 4, hipMemcpyDeviceToHost) != hipSuccess))
            st = set_error(MB_ERR_HIP, "mb_small_geneig: download failed");
        else if (status)
            st = set_error(MB_ERR_NONFINITE, "mb_small_geneig: non-finite input or result");
    }
    cleanup();
    return st;
}
