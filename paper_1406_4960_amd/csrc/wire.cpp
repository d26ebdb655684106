// Host set-up of the 1D-periodic form (B-splines along x and z, plane waves along the
// period in y): both spline directions, the plane-wave sets per k-point, the projector
// factors F_p(G) X_p(i) Z_p(j), and the z-direction eigenvectors of D_z u = lambda S_z u
// used by the eigensolver's preconditioner.  FP64, once per geometry.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "mbks_internal.h"

namespace mb {

namespace {

constexpr double kPi = 3.14159265358979323846;

// transform lengths with a compiled kernel
bool wire_ny_supported(int ny) {
    switch (ny) {
        case 8: case 12: case 16: case 24: case 32: case 48: case 64: case 128: return true;
        default: return false;
    }
}

// Projector factor of one direction, sum_q w_q B_i(x_q) f(x_q - X) with
// f = exp(-a u^2) (times u for the projector that is odd along this direction);
// rows outside the window of non-negligible values become exact zeros.
void projector_factor_1d(const SplineDir& d, double X0, double a, bool odd, double* row, int32_t* win) {
    const int K = 4;
    std::fill(row, row + d.nb, 0.0);
    for (int s = 0; s < d.nint; ++s)
        for (int j = 0; j < d.nq; ++j) {
            const int q = s * d.nq + j;
            const double u = d.zq[q] - X0;
            double f = std::exp(-a * u * u);
            if (odd) f *= u;
            for (int r = 0; r < K; ++r) {
                const int i = s - 1 + r;
                if (i < 0 || i >= d.nb) continue;
                row[i] += d.wbval[(size_t)q * K + r] * f;
            }
        }
    double mx = 0.0;
    for (int i = 0; i < d.nb; ++i) mx = std::max(mx, std::fabs(row[i]));
    int lo = d.nb, hi = -1;
    for (int i = 0; i < d.nb; ++i)
        if (std::fabs(row[i]) > 1e-16 * mx) { lo = std::min(lo, i); hi = std::max(hi, i); }
    if (hi < 0) { lo = 0; hi = -1; }
    for (int i = 0; i < d.nb; ++i)
        if (i < lo || i > hi) row[i] = 0.0;
    win[0] = lo;
    win[1] = hi;
}

// Symmetric eigenproblem A v = lambda v (n x n row-major, overwritten) by cyclic Jacobi
// rotations; V receives the eigenvectors as columns.
void jacobi_eigen(int n, std::vector<double>& A, std::vector<double>& V, std::vector<double>& lam) {
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    auto at = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) (i == j ? dia : off) += at(i, j) * at(i, j);
        if (off <= 1e-30 * dia) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = at(p, q);
                if (std::fabs(apq) < 1e-300) continue;
                const double theta = (at(q, q) - at(p, p)) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < n; ++k) {  // columns p, q
                    const double akp = at(k, p), akq = at(k, q);
                    at(k, p) = c * akp - sn * akq;
                    at(k, q) = sn * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // rows p, q
                    const double apk = at(p, k), aqk = at(q, k);
                    at(p, k) = c * apk - sn * aqk;
                    at(q, k) = sn * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - sn * vkq;
                    V[(size_t)k * n + q] = sn * vkp + c * vkq;
                }
            }
    }
    lam.resize(n);
    for (int i = 0; i < n; ++i) lam[i] = at(i, i);
}

// D u = lambda S u for banded S (Cholesky band L) and D: A = L^{-1} D L^{-T}, Jacobi,
// U = L^{-T} V (U^T S U = I, U^T D U = diag(lambda)).  U[j][j'] = component j of vector j'.
void banded_geneig(const SplineDir& d, std::vector<double>& U, std::vector<double>& lam) {
    const int n = d.nb, K = 4;
    auto Lb = [&](int i, int j) -> double {  // L[i][j], j <= i
        return (i - j < K && i >= j) ? d.lband[(size_t)i * K + (i - j)] : 0.0;
    };
    std::vector<double> D((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int dd = 0; dd < K && i + dd < n; ++dd) {
            D[(size_t)i * n + i + dd] = d.dband[(size_t)i * K + dd];
            D[(size_t)(i + dd) * n + i] = d.dband[(size_t)i * K + dd];
        }
    // B = L^{-1} D (forward substitution on every column), then A = B L^{-T} = (L^{-1} B^T)^T
    auto fwd = [&](std::vector<double>& M) {
        for (int c = 0; c < n; ++c)
            for (int i = 0; i < n; ++i) {
                double v = M[(size_t)i * n + c];
                for (int j = std::max(0, i - K + 1); j < i; ++j) v -= Lb(i, j) * M[(size_t)j * n + c];
                M[(size_t)i * n + c] = v / Lb(i, i);
            }
    };
    fwd(D);
    std::vector<double> A((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) A[(size_t)i * n + j] = D[(size_t)j * n + i];
    fwd(A);
    for (int i = 0; i < n; ++i)  // symmetrise rounding
        for (int j = i + 1; j < n; ++j) {
            const double v = 0.5 * (A[(size_t)i * n + j] + A[(size_t)j * n + i]);
            A[(size_t)i * n + j] = A[(size_t)j * n + i] = v;
        }
    std::vector<double> V;
    jacobi_eigen(n, A, V, lam);
    // U = L^{-T} V: back substitution on every column
    U = V;
    for (int c = 0; c < n; ++c)
        for (int i = n - 1; i >= 0; --i) {
            double v = U[(size_t)i * n + c];
            for (int j = i + 1; j < std::min(n, i + K); ++j) v -= Lb(j, i) * U[(size_t)j * n + c];
            U[(size_t)i * n + c] = v / Lb(i, i);
        }
}

}  // namespace

mb_status build_wire(const mb_wire_desc* d, Problem* p) {
    if (!d) return set_error(MB_ERR_INVALID_ARG, "desc is NULL");
    if (!(d->period > 0) || !std::isfinite(d->period)) return set_error(MB_ERR_INVALID_ARG, "period must be > 0");
    if (d->order != 4) return set_error(MB_ERR_INVALID_ARG, "the 1D-periodic form supports order 4 only");
    if (d->nbreak_x < 2 || !d->breakpoints_x || d->nbreak_z < 2 || !d->breakpoints_z)
        return set_error(MB_ERR_INVALID_ARG, "need >= 2 breakpoints along x and z");
    if (d->nq < 1 || d->nq > 8) return set_error(MB_ERR_INVALID_ARG, "nq must be 1..8");
    if (!wire_ny_supported(d->ny))
        return set_error(MB_ERR_INVALID_ARG, "ny must be 8, 12, 16, 24, 32, 48, 64 or 128");
    if (!(d->ecut > 0)) return set_error(MB_ERR_INVALID_ARG, "ecut must be > 0");
    if (d->nk < 1 || !d->kfrac) return set_error(MB_ERR_INVALID_ARG, "need >= 1 k-point");
    if (d->natoms < 0 || (d->natoms > 0 && !d->atoms)) return set_error(MB_ERR_INVALID_ARG, "atoms");
    if (d->nspecies < 0 || (d->nspecies > 0 && !d->species)) return set_error(MB_ERR_INVALID_ARG, "species");
    for (int j = 1; j < d->nbreak_x; ++j)
        if (!(d->breakpoints_x[j] > d->breakpoints_x[j - 1]))
            return set_error(MB_ERR_INVALID_ARG, "breakpoints_x must be strictly increasing");
    for (int j = 1; j < d->nbreak_z; ++j)
        if (!(d->breakpoints_z[j] > d->breakpoints_z[j - 1]))
            return set_error(MB_ERR_INVALID_ARG, "breakpoints_z must be strictly increasing");
    p->species.assign(d->species, d->species + d->nspecies);
    p->atoms.assign(d->atoms, d->atoms + d->natoms);
    for (const auto& a : p->atoms)
        if (a.species < 0 || a.species >= d->nspecies)
            return set_error(MB_ERR_INVALID_ARG, "atom species index out of range");
    for (const auto& s : p->species) {
        if (s.ngauss < 0 || s.ngauss > MB_MAX_GAUSS) return set_error(MB_ERR_INVALID_ARG, "ngauss");
        for (int t = 0; t < s.ngauss; ++t)
            if (!(s.gauss_w[t] > 0)) return set_error(MB_ERR_INVALID_ARG, "gaussian width <= 0");
        if (s.nonlocal && !(s.alpha_s > 0 && s.alpha_p > 0))
            return set_error(MB_ERR_INVALID_ARG, "projector exponents must be > 0");
        if (s.nonlocal && (s.q_s != 0.0 || s.q_p != 0.0))
            return set_error(MB_ERR_INVALID_ARG, "augmentation charges are not supported in the 1D-periodic form");
    }

    auto* w = new WireTables;
    p->wire = w;
    w->period = d->period;
    w->ny = d->ny;
    MB_TRY(build_spline_dir(std::vector<double>(d->breakpoints_x, d->breakpoints_x + d->nbreak_x), 4, d->nq, &w->x,
                            "overlap S_x"));
    MB_TRY(build_spline_dir(std::vector<double>(d->breakpoints_z, d->breakpoints_z + d->nbreak_z), 4, d->nq, &w->z,
                            "overlap S_z"));
    p->order = 4;
    p->nq = d->nq;
    p->nint = w->z.nint;
    p->nzq = w->z.nzq;
    p->nb = w->x.nb * w->z.nb;
    p->N1 = d->ny;
    p->N2 = 1;
    p->kfrac.assign(2 * (size_t)d->nk, 0.0);
    for (int ik = 0; ik < d->nk; ++ik) p->kfrac[2 * ik] = d->kfrac[ik];

    // projectors: x and z factors (every k), energies
    p->np = 0;
    for (const auto& a : p->atoms)
        if (p->species[a.species].nonlocal) p->np += 4;
    const int np = p->np, nbx = w->x.nb, nbz = w->z.nb;
    w->Xp.assign((size_t)np * nbx, 0.0);
    w->Zp.assign((size_t)np * nbz, 0.0);
    w->xwin.assign((size_t)np * 2, 0);
    w->zwin.assign((size_t)np * 2, 0);
    p->Ep.assign(np, 0.0);
    p->Qp.assign(np, 0.0);
    {
        int pidx = 0;
        for (const auto& a : p->atoms) {
            const mb_species& sp = p->species[a.species];
            if (!sp.nonlocal) continue;
            for (int t = 0; t < 4; ++t, ++pidx) {  // s, p_x, p_y, p_z
                const double al = t == 0 ? sp.alpha_s : sp.alpha_p;
                p->Ep[pidx] = t == 0 ? sp.E_s : sp.E_p;
                projector_factor_1d(w->x, a.pos[0], al, t == 1, &w->Xp[(size_t)pidx * nbx], &w->xwin[2 * pidx]);
                projector_factor_1d(w->z, a.pos[2], al, t == 3, &w->Zp[(size_t)pidx * nbz], &w->zwin[2 * pidx]);
            }
        }
    }
    // per x row, the projectors whose x window holds it
    w->ploff.assign(nbx + 1, 0);
    w->plist.clear();
    for (int i = 0; i < nbx; ++i) {
        w->ploff[i] = (int32_t)w->plist.size();
        for (int q = 0; q < np; ++q)
            if (w->xwin[2 * q] <= i && i <= w->xwin[2 * q + 1] && w->zwin[2 * q] <= w->zwin[2 * q + 1])
                w->plist.push_back(q);
    }
    w->ploff[nbx] = (int32_t)w->plist.size();

    banded_geneig(w->z, w->Uz, w->lamz);

    // plane-wave sets
    const double L = d->period;
    p->kp.assign(d->nk, KPoint{});
    for (int ik = 0; ik < d->nk; ++ik) {
        KPoint& kp = p->kp[ik];
        const double k = 2.0 * kPi * d->kfrac[ik] / L;
        const int nmax = (int)std::ceil(std::sqrt(2.0 * d->ecut) * L / (2.0 * kPi)) + 2;
        std::vector<int> ms;
        for (int m = -nmax; m <= nmax; ++m) {
            const double q = k + 2.0 * kPi * m / L;
            if (0.5 * q * q <= d->ecut) ms.push_back(m);
        }
        if (ms.empty()) return set_error(MB_ERR_INVALID_ARG, "empty plane-wave set");
        int mmax = 0;
        for (int m : ms) mmax = std::max(mmax, std::abs(m));
        if (2 * mmax + 1 > d->ny)
            return set_error(MB_ERR_INVALID_ARG, "plane-wave set does not fit the y transform (2 m_max + 1 > ny)");
        kp.ng = (int)ms.size();
        kp.ld = recommended_ld(kp.ng);
        kp.m.assign(2 * (size_t)kp.ng, 0);
        kp.kg.assign(2 * (size_t)kp.ng, 0.0);
        kp.kg2.resize(kp.ng);
        kp.gmap.resize(kp.ng);
        kp.gtab.assign(d->ny, -1);
        for (int g = 0; g < kp.ng; ++g) {
            const double q = k + 2.0 * kPi * ms[g] / L;
            kp.m[2 * g] = ms[g];
            kp.kg[2 * g] = q;
            kp.kg2[g] = q * q;
            const int n = ((ms[g] % d->ny) + d->ny) % d->ny;
            kp.gmap[g] = n;
            kp.gtab[n] = g;
        }
        // F_p(G) = C L^{-1/2} e^{-i q Y} sqrt(pi/a) e^{-q^2/4a} (x -i q / 2a for p_y)
        kp.F.assign((size_t)np * kp.ld, zd(0.0, 0.0));
        int pidx = 0;
        for (const auto& a : p->atoms) {
            const mb_species& sp = p->species[a.species];
            if (!sp.nonlocal) continue;
            const double cs = std::pow(2.0 * sp.alpha_s / kPi, 0.75);
            const double cp = std::pow(2.0 * sp.alpha_p / kPi, 0.75) * 2.0 * std::sqrt(sp.alpha_p);
            for (int t = 0; t < 4; ++t, ++pidx) {
                const double al = t == 0 ? sp.alpha_s : sp.alpha_p;
                const double c = (t == 0 ? cs : cp) / std::sqrt(L);
                for (int g = 0; g < kp.ng; ++g) {
                    const double q = kp.kg[2 * g];
                    const double gauss = std::sqrt(kPi / al) * std::exp(-q * q / (4.0 * al));
                    const zd phase(std::cos(-q * a.pos[1]), std::sin(-q * a.pos[1]));
                    const zd f = t == 2 ? zd(0.0, -q / (2.0 * al) * gauss) : zd(gauss, 0.0);
                    kp.F[(size_t)pidx * kp.ld + g] = c * phase * f;
                }
            }
        }
    }
    return MB_OK;
}

}  // namespace mb
