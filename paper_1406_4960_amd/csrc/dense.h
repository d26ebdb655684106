// Launchers of the dense kernels used by the eigensolver (FP64 vectors).
#pragma once

#include "mbks_internal.h"

namespace mb {

// C_z = A_z^H B_z with A_z, B_z given by pointer tables (z-major), K elements per vector.
// herm: the caller knows C_z is Hermitian (A^H H A, A^H S A); the wide matrix-core path then
// computes the upper tiles only and fills the rest by conjugation.
mb_status dense_gram(const void* const* ta, const void* const* tb, int MA, int NB, int nz, int64_t K, void* out,
                     void* scratch, size_t scratch_bytes, hipStream_t s, bool herm = false);
// Y_{z,n} = alpha sum_m W_z[m][n] X_{z,m} + beta Y_{z,n}; W_z is MI x NO row-major.
// low: the wide combinations may run with FP32 matrix-core arithmetic (reduced-precision
// cycles of the eigensolver)
mb_status dense_combo(const void* const* tx, void* const* ty, const void* W, int MI, int NO, int nz, int64_t K,
                      double alpha, double beta, hipStream_t s, bool low = false);
// scratch: at least 64 * nvec complex doubles
mb_status dense_dots(const void* const* ta, const void* const* tb, int nvec, int64_t K, void* out, void* scratch,
                     hipStream_t s);
mb_status dense_resid(const void* const* th, const void* const* ts, const double* theta, int nvec, int64_t K,
                      double* out, hipStream_t s);
mb_status dense_axpy(void* const* ty, const void* const* tx, const void* coef, double sign, int nvec, int64_t K,
                     hipStream_t s);
mb_status dense_normalize(void* const* t1, void* const* t2, const void* d, int nvec, int64_t K, hipStream_t s);
mb_status dense_random(void* x, int nvec, int nb, int ld, int ng, uint64_t seed, hipStream_t s);
// nz problems of size N: H, S, Y row-major N x N each, evals N each; gwork of
// geneig_work_bytes(N, nz) bytes.  Problems whose work matrices do not fit in LDS
// synchronize the stream once per Jacobi sweep (the host reads a convergence flag).
size_t geneig_work_bytes(int N, int nz);
mb_status dense_geneig(const void* H, const void* S, int N, int nz, double* evals, void* Y, void* gwork,
                       int* status, hipStream_t s, int* sweeps = nullptr);
// map (device, nblocks entries, or null): block z's roots go to theta[map[z] * b + a]
mb_status dense_select(const void* Y, const double* ev, int nr, int b, void* C, double* theta, int nblocks,
                       hipStream_t s, const int32_t* map = nullptr);
// dst[v] = src[v] (K elements each) for the n vectors of two device pointer tables
mb_status dense_copy_tab(void* const* dst, const void* const* src, int n, int64_t K, hipStream_t s);
mb_status dense_copy_cols(const void* Y, int ldy, int ncols, int nrows, void* out, hipStream_t s);

}  // namespace mb
