// Generalized Lanczos-Krylov eigensolver (Sec. II.C) for H c = eps S c.
//
// The two grand cycles of the method alternate:
//  (B) block cycle: the trial vectors are split into blocks of `block`
//      consecutive roots; every block is diagonalised in the span of its own
//      vectors and a Krylov subspace of depth `krylov` grown from the block
//      member with the largest residual.  All blocks advance together, so each
//      Krylov step is one H application to nblocks vectors.  Krylov vectors are
//      S-orthogonalised (Gram-Schmidt, twice) against all trial vectors and the
//      block's earlier Krylov vectors.  Roots are chosen by maximum overlap with
//      the block's input vectors; lower unmatched roots of the block are picked
//      up as new roots.
//  (A) global cycle: Rayleigh-Ritz over the union of all trial vectors and a
//      Krylov subspace of depth `krylov_global` grown from the trial vector with
//      the largest residual; the nev lowest roots are kept.
// Every projected matrix is diagonalised by the cyclic Jacobi method after a
// Cholesky reduction of its overlap.  The Krylov sequence is generated with the
// preconditioned shifted operator K (H - theta S), K = (T + sigma S)^{-1}
// per G (or S^{-1} for sigma <= 0, which spans the same space as repeated
// S^{-1} H).  Orthonormalisation, recurrence coefficients and projected
// problems are FP64; reduced precision only enters H applications.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "dense.h"
#include "mbks_internal.h"

namespace mb {

Problem* problem_of(mb_problem* h);

namespace {

#define LZ_TRY(call)                \
    do {                            \
        mb_status s_ = (call);      \
        if (s_ != MB_OK) return s_; \
    } while (0)

struct Solver {
    Problem* p;
    int ik;
    hipStream_t s;
    int M, b, nbl, m, mA, NG, NR;
    int nwant;  // leading vectors whose residuals decide convergence (the rest are buffer)
    int ld;
    int64_t K;  // complex elements per vector
    size_t vbytes;
    // vectors
    char* X;
    char* HX;
    char* SX;
    char* Xn;
    char* HXn;
    char* SXn;
    char* Kv;
    char* HK;
    char* SK;
    // device tables
    void** tX;
    void** tHX;
    void** tSX;
    void** tXn;
    void** tHXn;
    void** tSXn;
    void** tK;
    void** tHK;
    void** tSK;
    void** tQ;
    void** tHQ;
    void** tSQ;
    // per Krylov depth j >= 1: block-batched Gram-Schmidt tables (see orthonormalise_k)
    std::vector<void**> tGA, tGB, tGX, tGO;
    void* dscratch;
    // soft locking: active block count of the current block cycle, the residual at or
    // below which a block sits out, per-cycle tables of a partial block set
    int na = 0;
    double lock_tol = 0.0;
    void** tpart;
    int32_t* amap;
    std::vector<void*> h_ptab;
    // small device arrays
    void* Hp;
    void* Sp;
    void* Y;
    void* W;
    void* gwork;
    double* evals;
    void* coef;
    void* dots;
    double* theta;
    double* theta_s;
    int32_t* sel;
    double* resid;
    int* status;
    void* gscratch;
    size_t gscratch_bytes;
    // host mirrors
    std::vector<double> h_theta, h_resid;
    int64_t applies = 0, applies_low = 0;
    // combinations of the current cycle may use FP32 matrix cores (Gram products stay in
    // FP64: the projected problems need their overlap to FP64 accuracy)
    bool low = false;

    char* vec(char* base, int i) const { return base + (size_t)i * vbytes; }

    mb_status hop(const void* c, void* y, void* sy, int n, int prec) {
        LZ_TRY(apply_h(p, ik, c, y, sy, n, ld, prec, s));
        applies += n;
        if (prec != 0) applies_low += n;
        return MB_OK;
    }

    mb_status check_status() {
        int st = 0;
        MB_HIP_TRY(hipMemcpyAsync(&st, status, sizeof(int), hipMemcpyDeviceToHost, s));
        MB_HIP_TRY(hipStreamSynchronize(s));
        if (st != 0) return set_error(MB_ERR_NONFINITE, "non-finite value in a projected eigenproblem");
        return MB_OK;
    }

    // global Rayleigh-Ritz over the first n vectors of X (n = M or NG): keep M lowest
    mb_status global_rr(int n) {
        // X^H H X and X^H S X are Hermitian: the matrix-core path computes half of each
        LZ_TRY(dense_gram((const void* const*)tX, (const void* const*)tHX, n, n, 1, K, Hp, gscratch, gscratch_bytes, s,
                          true));
        LZ_TRY(dense_gram((const void* const*)tX, (const void* const*)tSX, n, n, 1, K, Sp, gscratch, gscratch_bytes, s,
                          true));
        LZ_TRY(dense_geneig(Hp, Sp, n, 1, evals, Y, gwork, status, s));
        LZ_TRY(dense_copy_cols(Y, n, M, n, W, s));
        LZ_TRY(dense_combo((const void* const*)tX, tXn, W, n, M, 1, K, 1.0, 0.0, s, low));
        LZ_TRY(dense_combo((const void* const*)tHX, tHXn, W, n, M, 1, K, 1.0, 0.0, s, low));
        LZ_TRY(dense_combo((const void* const*)tSX, tSXn, W, n, M, 1, K, 1.0, 0.0, s, low));
        MB_HIP_TRY(hipMemcpyAsync(X, Xn, (size_t)M * vbytes, hipMemcpyDeviceToDevice, s));
        MB_HIP_TRY(hipMemcpyAsync(HX, HXn, (size_t)M * vbytes, hipMemcpyDeviceToDevice, s));
        MB_HIP_TRY(hipMemcpyAsync(SX, SXn, (size_t)M * vbytes, hipMemcpyDeviceToDevice, s));
        MB_HIP_TRY(hipMemcpyAsync(theta, evals, (size_t)M * sizeof(double), hipMemcpyDeviceToDevice, s));
        return check_status();
    }

    mb_status residuals() {
        LZ_TRY(dense_resid((const void* const*)tHX, (const void* const*)tSX, theta, M, K, resid, s));
        MB_HIP_TRY(hipMemcpyAsync(h_resid.data(), resid, M * sizeof(double), hipMemcpyDeviceToHost, s));
        MB_HIP_TRY(hipMemcpyAsync(h_theta.data(), theta, M * sizeof(double), hipMemcpyDeviceToHost, s));
        MB_HIP_TRY(hipStreamSynchronize(s));
        for (int j = 0; j < M; ++j)
            if (!std::isfinite(h_resid[j]) || !std::isfinite(h_theta[j]))
                return set_error(MB_ERR_NONFINITE, "non-finite residual or eigenvalue");
        return MB_OK;
    }

    // S-orthonormalise Krylov slot j (the na active blocks) against X[0..M) and, block by
    // block, against the block's K[0..j): classical Gram-Schmidt, two passes.  In the
    // reduced-precision cycles of a mixed solve one pass: their H applications and
    // combinations carry FP32 rounding anyway, and the Rayleigh-Ritz steps that follow
    // take the overlap of whatever subspace results in FP64 (measured on the 128x64
    // surface slab, 320 roots: the same cycle count, eigenvalues within 4e-15 Ha of the
    // two-pass solve, 13 % less time)
    mb_status orthonormalise_k(int j) {
        void** tKj = tK + (size_t)j * nbl;
        void** tSKj = tSK + (size_t)j * nbl;
        char* Kj = vec(Kv, j * nbl);
        char* SKj = vec(SK, j * nbl);
        const int passes = low ? 1 : 2;
        for (int pass = 0; pass < passes; ++pass) {
            // against all trial vectors: C = (S X)^H K_j, K_j -= X C
            LZ_TRY(dense_gram((const void* const*)tSX, (const void* const*)tKj, M, na, 1, K, coef, gscratch,
                              gscratch_bytes, s));
            LZ_TRY(dense_combo((const void* const*)tX, tKj, coef, M, na, 1, K, -1.0, 1.0, s, low));
            if (j > 0) {
                // d[z*j + i] = <K_i^z|S|K_j^z>, then K_j^z -= sum_i d[z*j + i] K_i^z
                LZ_TRY(dense_dots((const void* const*)tGA[j], (const void* const*)tGB[j], na * j, K, dots,
                                  dscratch, s));
                LZ_TRY(dense_combo((const void* const*)tGX[j], tGO[j], dots, j, 1, na, K, -1.0, 1.0, s));
            }
        }
        LZ_TRY(launch_spsi(p, ik, Kj, SKj, na, ld, 0, s));
        LZ_TRY(dense_dots((const void* const*)tKj, (const void* const*)tSKj, na, K, dots, dscratch, s));
        LZ_TRY(dense_normalize(tKj, tSKj, dots, na, K, s));
        return MB_OK;
    }

    // Soft locking: a block whose members all have residuals at or below lock_tol sits
    // out the block cycle (no Krylov vectors, no block Rayleigh-Ritz); its trial vectors
    // stay in X and in the global Rayleigh-Ritz step, and the block rejoins as soon as
    // a residual rises above lock_tol again.  The na active blocks take Krylov slots
    // 0..na-1, so every per-slot table and the contiguous H applications keep their
    // layout; the block Rayleigh-Ritz step of a partial set runs on tables built here.
    mb_status block_cycle(int prec) {
        // active blocks and their seeds (the member with the largest residual)
        std::vector<int32_t> seeds, act;
        std::vector<double> th;
        for (int z = 0; z < nbl; ++z) {
            int best = z * b;
            for (int a = 1; a < b; ++a)
                if (h_resid[z * b + a] > h_resid[best]) best = z * b + a;
            if (!(h_resid[best] > lock_tol)) continue;
            act.push_back(z);
            seeds.push_back(best);
            th.push_back(h_theta[best]);
        }
        na = (int)act.size();
        if (na == 0) return MB_OK;
        MB_HIP_TRY(hipMemcpyAsync(sel, seeds.data(), na * sizeof(int32_t), hipMemcpyHostToDevice, s));
        MB_HIP_TRY(hipMemcpyAsync(theta_s, th.data(), na * sizeof(double), hipMemcpyHostToDevice, s));
        const bool part = na < nbl;
        if (part) {
            // block Rayleigh-Ritz tables of the active blocks: Q = [x_z members, K_0..K_{m-1}]
            // (K of active block i in slot position i), outputs and copy targets at the
            // blocks' own trial-vector positions
            h_ptab.clear();
            for (int which = 0; which < 3; ++which) {
                char* xb = which == 0 ? X : which == 1 ? HX : SX;
                char* kb = which == 0 ? Kv : which == 1 ? HK : SK;
                for (int i = 0; i < na; ++i) {
                    for (int a = 0; a < b; ++a) h_ptab.push_back(xb + (size_t)(act[i] * b + a) * vbytes);
                    for (int j = 0; j < m; ++j) h_ptab.push_back(kb + (size_t)(j * nbl + i) * vbytes);
                }
            }
            for (int which = 0; which < 6; ++which) {
                char* vb = which == 0 ? Xn : which == 1 ? HXn : which == 2 ? SXn : which == 3 ? X : which == 4 ? HX : SX;
                for (int i = 0; i < na; ++i)
                    for (int a = 0; a < b; ++a) h_ptab.push_back(vb + (size_t)(act[i] * b + a) * vbytes);
            }
            MB_HIP_TRY(hipMemcpyAsync(tpart, h_ptab.data(), h_ptab.size() * sizeof(void*), hipMemcpyHostToDevice, s));
            MB_HIP_TRY(hipMemcpyAsync(amap, act.data(), na * sizeof(int32_t), hipMemcpyHostToDevice, s));
        }
        MB_HIP_TRY(hipStreamSynchronize(s));
        // K_1 = P (H x_s - theta_s S x_s)
        LZ_TRY(launch_prec_apply(p, ik, HX, SX, theta_s, sel, vec(Kv, 0), na, ld, s));
        for (int j = 0; j < m; ++j) {
            LZ_TRY(orthonormalise_k(j));
            LZ_TRY(hop(vec(Kv, j * nbl), vec(HK, j * nbl), nullptr, na, prec));
            if (j + 1 < m)
                LZ_TRY(launch_prec_apply(p, ik, vec(HK, j * nbl), vec(SK, j * nbl), theta_s, nullptr,
                                         vec(Kv, (j + 1) * nbl), na, ld, s));
        }
        // per-block Rayleigh-Ritz
        const size_t qn = (size_t)na * NR, on = (size_t)na * b;
        void** q = part ? tpart : tQ;
        void** hq = part ? tpart + qn : tHQ;
        void** sq = part ? tpart + 2 * qn : tSQ;
        void** xo = part ? tpart + 3 * qn : tXn;
        void** hxo = part ? tpart + 3 * qn + on : tHXn;
        void** sxo = part ? tpart + 3 * qn + 2 * on : tSXn;
        LZ_TRY(dense_gram((const void* const*)q, (const void* const*)hq, NR, NR, na, K, Hp, gscratch, gscratch_bytes, s));
        LZ_TRY(dense_gram((const void* const*)q, (const void* const*)sq, NR, NR, na, K, Sp, gscratch, gscratch_bytes, s));
        LZ_TRY(dense_geneig(Hp, Sp, NR, na, evals, Y, gwork, status, s));
        LZ_TRY(dense_select(Y, evals, NR, b, W, theta, na, s, part ? amap : nullptr));
        LZ_TRY(dense_combo((const void* const*)q, xo, W, NR, b, na, K, 1.0, 0.0, s));
        LZ_TRY(dense_combo((const void* const*)hq, hxo, W, NR, b, na, K, 1.0, 0.0, s));
        LZ_TRY(dense_combo((const void* const*)sq, sxo, W, NR, b, na, K, 1.0, 0.0, s));
        if (part) {
            LZ_TRY(dense_copy_tab(tpart + 3 * qn + 3 * on, (const void* const*)(tpart + 3 * qn), 3 * (int)on, K, s));
        } else {
            MB_HIP_TRY(hipMemcpyAsync(X, Xn, (size_t)M * vbytes, hipMemcpyDeviceToDevice, s));
            MB_HIP_TRY(hipMemcpyAsync(HX, HXn, (size_t)M * vbytes, hipMemcpyDeviceToDevice, s));
            MB_HIP_TRY(hipMemcpyAsync(SX, SXn, (size_t)M * vbytes, hipMemcpyDeviceToDevice, s));
        }
        return check_status();
    }

    mb_status global_cycle(int prec) {
        if (mA == 0) return global_rr(M);
        int v = 0;
        for (int j = 1; j < nwant; ++j)
            if (h_resid[j] > h_resid[v]) v = j;
        // Krylov vectors in X[M .. M+mA)
        LZ_TRY(launch_prec_apply(p, ik, vec(HX, v), vec(SX, v), theta + v, nullptr, vec(X, M), 1, ld, s));
        for (int j = 0; j < mA; ++j) {
            int slot = M + j;
            for (int pass = 0; pass < 2; ++pass)
                for (int i = 0; i < j; ++i) {
                    LZ_TRY(dense_dots((const void* const*)(tSX + M + i), (const void* const*)(tX + slot), 1, K, dots,
                                      dscratch, s));
                    LZ_TRY(dense_axpy(tX + slot, (const void* const*)(tX + M + i), dots, -1.0, 1, K, s));
                }
            LZ_TRY(launch_spsi(p, ik, vec(X, slot), vec(SX, slot), 1, ld, 0, s));
            LZ_TRY(dense_dots((const void* const*)(tX + slot), (const void* const*)(tSX + slot), 1, K, dots, dscratch,
                              s));
            LZ_TRY(dense_normalize(tX + slot, tSX + slot, dots, 1, K, s));
            LZ_TRY(hop(vec(X, slot), vec(HX, slot), nullptr, 1, prec));
            if (j + 1 < mA)
                LZ_TRY(launch_prec_apply(p, ik, vec(HX, slot), vec(SX, slot), theta + v, nullptr, vec(X, slot + 1), 1,
                                         ld, s));
        }
        return global_rr(NG);
    }
};

}  // namespace

// Shape of one solve: M iterated vectors (nev wanted + buffer), nbl blocks of b, Krylov
// depth m, global Krylov depth mA.
struct LzShape {
    int M, b, nbl, m, mA;
};

static LzShape lz_shape(const Problem* p, int ik, int nev, const mb_lanczos_opts& o) {
    const int64_t basis = (int64_t)p->kp[ik].ng * p->nb;
    int nbuf = o.extra >= 0 ? o.extra : std::min(16, std::max(4, nev / 4));
    nbuf = (int)std::max<int64_t>(0, std::min<int64_t>(nbuf, basis - nev));
    LzShape z{};
    z.M = nev + nbuf;
    z.b = std::max(1, std::min(o.block, z.M));
    while (z.M % z.b) --z.b;
    z.nbl = z.M / z.b;
    z.m = std::max(1, o.krylov);
    z.mA = std::max(0, o.krylov_global);
    return z;
}

// Vector workspace of one solve: trial vectors X, HX, SX (M + mA), their rotation
// targets (M), and the block Krylov vectors K, HK, SK (m per block), all complex128.
size_t lanczos_vector_bytes(const Problem* p, int ik, int nev, const mb_lanczos_opts& o) {
    const LzShape z = lz_shape(p, ik, nev, o);
    const size_t nvec = 3 * (size_t)(z.M + z.mA) + 3 * (size_t)z.M + 3 * (size_t)z.m * z.nbl;
    return nvec * (size_t)p->nb * p->kp[ik].ld * 16;
}

// Device memory a solve holds at its peak: the vectors above and the partial rows and
// projector partials of FP64 H applications to M vectors at once (the widest ones).
size_t lanczos_device_bytes(const Problem* p, int ik, int nev, const mb_lanczos_opts& o) {
    const KPoint& kp = p->kp[ik];
    const LzShape z = lz_shape(p, ik, nev, o);
    const size_t h = (size_t)std::max(z.M, z.nbl);
    const size_t part = h * (size_t)p->nint * 4 * kp.ld * 16;
    const size_t nl = (size_t)p->nb * ((p->np + 15) / 16 * 16) * ((h + 15) / 16 * 16) * 16;
    return lanczos_vector_bytes(p, ik, nev, o) + part + nl;
}

// a k-point keeps its eigensolver vectors between solves only up to this size; larger
// ones (hundreds of bands on large slabs) are released so that the solves of several
// k-points of one problem can follow each other on one GPU
constexpr size_t LZ_KEEP_BYTES = (size_t)8 << 30;

mb_status lanczos_impl(Problem* p, int ik, int nev, mb_precision prec, const mb_lanczos_opts& o, const void* x0,
                       double* eig, void* xout, mb_lanczos_info* info, hipStream_t s) {
    auto t0 = std::chrono::steady_clock::now();
    const KPoint& kp = p->kp[ik];
    Solver S{};
    S.p = p;
    S.ik = ik;
    S.s = s;
    // nbuf buffer vectors above the nev wanted ones: iterated like the others but not
    // required to converge, so a cluster straddling the nev-th root does not stall
    // the iteration
    const int64_t basis = (int64_t)kp.ng * p->nb;
    int nbuf = o.extra >= 0 ? o.extra : std::min(16, std::max(4, nev / 4));
    nbuf = (int)std::max<int64_t>(0, std::min<int64_t>(nbuf, basis - nev));
    const int M = nev + nbuf;
    S.M = M;
    S.nwant = nev;
    S.b = std::max(1, std::min(o.block, M));
    while (M % S.b) --S.b;
    S.nbl = M / S.b;
    S.m = std::max(1, o.krylov);
    S.mA = std::max(0, o.krylov_global);
    S.NG = M + S.mA;
    S.NR = S.b + S.m;
    S.ld = kp.ld;
    S.K = (int64_t)p->nb * kp.ld;
    S.vbytes = (size_t)S.K * 16;
    if (S.NG > 512 || S.NR > 64 || S.b > 32)
        return set_error(MB_ERR_INVALID_ARG,
                         "lanczos_lowest: nev + buffer + krylov_global must be <= 512, block + krylov <= 64");
    if ((int64_t)nev > basis) return set_error(MB_ERR_INVALID_ARG, "nev exceeds the basis size");

    // vector workspace
    size_t nvec = 3 * (size_t)S.NG + 3 * (size_t)S.M + 3 * (size_t)S.m * S.nbl;
    KPoint& kw = p->kp[ik];
    if (nvec * S.vbytes != lanczos_vector_bytes(p, ik, nev, o))
        return set_error(MB_ERR_INVALID_ARG, "lanczos_lowest: workspace size mismatch");
    LZ_TRY(ensure_ws(kw.ws_lz, nvec * S.vbytes));
    char* base = (char*)kw.ws_lz.ptr;
    auto take = [&](int n) {
        char* r = base;
        base += (size_t)n * S.vbytes;
        return r;
    };
    S.X = take(S.NG);
    S.HX = take(S.NG);
    S.SX = take(S.NG);
    S.Xn = take(S.M);
    S.HXn = take(S.M);
    S.SXn = take(S.M);
    S.Kv = take(S.m * S.nbl);
    S.HK = take(S.m * S.nbl);
    S.SK = take(S.m * S.nbl);

    // small workspace
    const size_t NN = std::max((size_t)S.NG * S.NG, (size_t)S.nbl * S.NR * S.NR);
    const size_t ntab = 3 * (size_t)S.NG + 3 * (size_t)S.M + 3 * (size_t)S.m * S.nbl + 3 * (size_t)S.nbl * S.NR +
                        (size_t)S.nbl * (3 * (size_t)S.m * S.m / 2 + S.m + 1);
    S.gscratch_bytes = std::max((size_t)32 << 20, 4 * NN * 16);  // Gram partial sums over k chunks
    size_t small = ntab * sizeof(void*) + 3 * NN * 16 + (size_t)S.NG * S.M * 16 + (size_t)S.nbl * S.NR * S.b * 16 +
                   4 * NN * 16 + 16 * (size_t)std::max(S.nbl, 1) + 64 + NN * sizeof(double) + (size_t)S.M * std::max(S.nbl, S.NG) * 16 +
                   (size_t)S.nbl * S.m * 16 + (size_t)64 * std::max(S.nbl * S.m, S.NG) * 16 +
                   (3 * (size_t)S.M + S.NG + 2 * S.nbl + 64) * 8 + S.gscratch_bytes + 64 * 256 +
                   ((size_t)3 * S.nbl * S.NR + (size_t)6 * S.M) * sizeof(void*) + (size_t)S.nbl * 4 + 512;
    LZ_TRY(ensure_ws(kw.ws_small, small));
    char* sb = (char*)kw.ws_small.ptr;
    auto stake = [&](size_t bytes) {
        char* r = sb;
        sb += (bytes + 255) / 256 * 256;
        return (void*)r;
    };
    std::vector<void*> htab;
    auto add_tab = [&](char* vbase, int n) {
        size_t off = htab.size();
        for (int i = 0; i < n; ++i) htab.push_back(vbase + (size_t)i * S.vbytes);
        return off;
    };
    size_t oX = add_tab(S.X, S.NG), oHX = add_tab(S.HX, S.NG), oSX = add_tab(S.SX, S.NG);
    size_t oXn = add_tab(S.Xn, S.M), oHXn = add_tab(S.HXn, S.M), oSXn = add_tab(S.SXn, S.M);
    size_t oK = add_tab(S.Kv, S.m * S.nbl), oHK = add_tab(S.HK, S.m * S.nbl), oSK = add_tab(S.SK, S.m * S.nbl);
    size_t oQ = htab.size();
    for (int which = 0; which < 3; ++which) {
        char* xb = which == 0 ? S.X : which == 1 ? S.HX : S.SX;
        char* kb = which == 0 ? S.Kv : which == 1 ? S.HK : S.SK;
        for (int z = 0; z < S.nbl; ++z) {
            for (int a = 0; a < S.b; ++a) htab.push_back(xb + (size_t)(z * S.b + a) * S.vbytes);
            for (int j = 0; j < S.m; ++j) htab.push_back(kb + (size_t)(j * S.nbl + z) * S.vbytes);
        }
    }
    std::vector<size_t> oGA(S.m, 0), oGB(S.m, 0), oGX(S.m, 0), oGO(S.m, 0);
    for (int j = 1; j < S.m; ++j) {
        oGA[j] = htab.size();
        for (int z = 0; z < S.nbl; ++z)
            for (int i = 0; i < j; ++i) htab.push_back(S.SK + (size_t)(i * S.nbl + z) * S.vbytes);
        oGB[j] = htab.size();
        for (int z = 0; z < S.nbl; ++z)
            for (int i = 0; i < j; ++i) htab.push_back(S.Kv + (size_t)(j * S.nbl + z) * S.vbytes);
        oGX[j] = htab.size();
        for (int z = 0; z < S.nbl; ++z)
            for (int i = 0; i < j; ++i) htab.push_back(S.Kv + (size_t)(i * S.nbl + z) * S.vbytes);
        oGO[j] = htab.size();
        for (int z = 0; z < S.nbl; ++z) htab.push_back(S.Kv + (size_t)(j * S.nbl + z) * S.vbytes);
    }
    void** dtab = (void**)stake(htab.size() * sizeof(void*));
    MB_HIP_TRY(hipMemcpyAsync(dtab, htab.data(), htab.size() * sizeof(void*), hipMemcpyHostToDevice, s));
    S.tX = dtab + oX; S.tHX = dtab + oHX; S.tSX = dtab + oSX;
    S.tXn = dtab + oXn; S.tHXn = dtab + oHXn; S.tSXn = dtab + oSXn;
    S.tK = dtab + oK; S.tHK = dtab + oHK; S.tSK = dtab + oSK;
    size_t qn = (size_t)S.nbl * S.NR;
    S.tQ = dtab + oQ; S.tHQ = dtab + oQ + qn; S.tSQ = dtab + oQ + 2 * qn;
    S.tGA.assign(S.m, nullptr); S.tGB.assign(S.m, nullptr); S.tGX.assign(S.m, nullptr); S.tGO.assign(S.m, nullptr);
    for (int j = 1; j < S.m; ++j) {
        S.tGA[j] = dtab + oGA[j]; S.tGB[j] = dtab + oGB[j]; S.tGX[j] = dtab + oGX[j]; S.tGO[j] = dtab + oGO[j];
    }
    S.Hp = stake(NN * 16);
    S.Sp = stake(NN * 16);
    S.Y = stake(NN * 16);
    S.W = stake(std::max((size_t)S.NG * S.M, (size_t)S.nbl * S.NR * S.b) * 16);
    S.gwork = stake(4 * NN * 16 + 16 * (size_t)std::max(S.nbl, 1) + 64);
    S.evals = (double*)stake(NN * sizeof(double));
    S.coef = stake((size_t)S.M * std::max(S.nbl, S.NG) * 16);
    S.dots = stake((size_t)std::max(S.nbl * S.m, 1) * 16);
    S.dscratch = stake((size_t)64 * std::max(S.nbl * S.m, S.NG) * 16);
    S.theta = (double*)stake(S.NG * sizeof(double));
    S.theta_s = (double*)stake(S.nbl * sizeof(double));
    S.sel = (int32_t*)stake(S.nbl * sizeof(int32_t));
    S.resid = (double*)stake(S.M * sizeof(double));
    S.status = (int*)stake(64);
    S.gscratch = stake(S.gscratch_bytes);
    S.tpart = (void**)stake(((size_t)3 * S.nbl * S.NR + (size_t)6 * S.M) * sizeof(void*));
    S.amap = (int32_t*)stake((size_t)S.nbl * sizeof(int32_t));
    S.na = S.nbl;
    S.lock_tol = o.tol;
    if ((size_t)(sb - (char*)kw.ws_small.ptr) > kw.ws_small.bytes) return set_error(MB_ERR_INVALID_ARG, "small workspace layout");
    MB_HIP_TRY(hipMemsetAsync(S.status, 0, sizeof(int), s));
    S.h_theta.assign(S.M, 0.0);
    S.h_resid.assign(S.M, 0.0);

    LZ_TRY(launch_prec_factor(p, ik, o.sigma, s));

    // start vectors
    if (x0) {
        MB_HIP_TRY(hipMemcpyAsync(S.X, x0, (size_t)nev * S.vbytes, hipMemcpyDeviceToDevice, s));
        if (nbuf > 0) LZ_TRY(dense_random(S.vec(S.X, nev), nbuf, p->nb, S.ld, kp.ng, o.seed, s));
    } else {
        LZ_TRY(dense_random(S.X, S.M, p->nb, S.ld, kp.ng, o.seed, s));
    }
    int cur = prec == MB_FP64 ? 0 : prec == MB_FP32 ? 2 : 4;
    const bool low_dense = o.dense_low != 0;
    S.low = cur != 0 && low_dense;
    LZ_TRY(S.hop(S.X, S.HX, S.SX, S.M, cur));
    LZ_TRY(S.global_rr(S.M));

    mb_status result = MB_ERR_NOT_CONVERGED;
    int it = 0, it_low = 0;
    double best = 1e300;
    int stall = 0;
    for (; it < o.max_iter; ++it) {
        LZ_TRY(S.residuals());
        double mx = *std::max_element(S.h_resid.begin(), S.h_resid.begin() + nev);
        if (cur != 0) {
            if (mx < 0.9 * best) { best = mx; stall = 0; } else ++stall;
            if (mx <= o.switch_tol || stall >= 4) {
                // continue in FP64: refresh H X at full precision
                cur = 0;
                S.low = false;
                LZ_TRY(S.hop(S.X, S.HX, S.SX, S.M, 0));
                LZ_TRY(S.global_rr(S.M));
                LZ_TRY(S.residuals());
                mx = *std::max_element(S.h_resid.begin(), S.h_resid.begin() + nev);
            }
        }
        if (cur == 0 && mx <= o.tol) {
            result = MB_OK;
            break;
        }
        if (cur != 0) ++it_low;
        LZ_TRY(S.block_cycle(cur));
        // residual estimates for the seed of the global cycle
        LZ_TRY(dense_resid((const void* const*)S.tHX, (const void* const*)S.tSX, S.theta, S.M, S.K, S.resid, s));
        MB_HIP_TRY(hipMemcpyAsync(S.h_resid.data(), S.resid, S.M * sizeof(double), hipMemcpyDeviceToHost, s));
        MB_HIP_TRY(hipStreamSynchronize(s));
        LZ_TRY(S.global_cycle(cur));
    }
    if (result != MB_OK) {
        LZ_TRY(S.residuals());
        set_error(MB_ERR_NOT_CONVERGED, "lanczos_lowest: max_iter reached");
    }
    if (xout) MB_HIP_TRY(hipMemcpyAsync(xout, S.X, (size_t)nev * S.vbytes, hipMemcpyDeviceToDevice, s));
    MB_HIP_TRY(hipStreamSynchronize(s));
    if (kw.ws_lz.bytes > LZ_KEEP_BYTES) {
        // with it go the H-application work buffers sized for this solve
        for (Workspace* w : {&kw.ws_lz, &kw.ws_part, &kw.ws_nlpart}) {
            if (kw.locked && w != &kw.ws_lz) continue;  // reserved H work buffers stay
            if (w->ptr) MB_HIP_TRY(hipFree(w->ptr));
            w->ptr = nullptr;
            w->bytes = 0;
        }
    }
    if (eig) std::memcpy(eig, S.h_theta.data(), nev * sizeof(double));
    if (info) {
        info->iters = it;
        info->iters_low = it_low;
        info->h_applies = S.applies;
        info->h_applies_low = S.applies_low;
        info->max_resid = *std::max_element(S.h_resid.begin(), S.h_resid.begin() + nev);
        info->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return result;
}

}  // namespace mb

extern "C" void mb_lanczos_default_opts(mb_lanczos_opts* o) {
    if (!o) return;
    o->block = 1;
    o->krylov = 4;
    o->krylov_global = 2;
    o->max_iter = 300;
    o->tol = 1e-7;
    o->sigma = 0.05;
    o->switch_tol = 1e-4;
    o->seed = 14064960ull;
    o->extra = -1;
    o->dense_low = 1;
}

extern "C" mb_status lanczos_lowest(mb_problem* h, int ik, int nev, mb_precision prec, const mb_lanczos_opts* opts,
                                    const void* x0, double* eig, void* x, mb_lanczos_info* info, void* stream) {
    mb::Problem* p = mb::problem_of(h);
    if (!p) return mb::set_error(MB_ERR_INVALID_ARG, "lanczos_lowest: problem is NULL");
    if (p->device < 0) return mb::set_error(MB_ERR_NO_DEVICE, "lanczos_lowest: host-only problem");
    if (ik < 0 || ik >= (int)p->kp.size()) return mb::set_error(MB_ERR_INVALID_ARG, "lanczos_lowest: ik out of range");
    if (nev < 1) return mb::set_error(MB_ERR_INVALID_ARG, "lanczos_lowest: nev < 1");
    if (prec != MB_FP64 && prec != MB_FP32 && prec != MB_BF16X3)
        return mb::set_error(MB_ERR_INVALID_ARG, "lanczos_lowest: unknown precision");
    if (p->order != 4) return mb::set_error(MB_ERR_INVALID_ARG, "lanczos_lowest: GPU kernels support order 4 only");
    mb_lanczos_opts o;
    mb_lanczos_default_opts(&o);
    if (opts) o = *opts;
    if (o.max_iter < 1 || o.krylov < 1 || o.block < 1 || o.krylov_global < 0 || !(o.tol > 0))
        return mb::set_error(MB_ERR_INVALID_ARG, "lanczos_lowest: bad options");
    return mb::lanczos_impl(p, ik, nev, prec, o, x0, eig, x, info, (hipStream_t)stream);
}
