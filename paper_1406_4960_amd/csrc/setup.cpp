// Host set-up of one problem: knots, Gauss rule, B-spline tables, banded 1D
// matrices and their Cholesky factor, G sets, grid maps and projector factors.
// Everything here runs once per geometry in FP64.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "mbks_internal.h"

namespace mb {

namespace {

constexpr double kPi = 3.14159265358979323846;

// Gauss-Legendre nodes and weights on [-1, 1]: Newton iteration on P_n from the
// Chebyshev-like initial guess, weights 2 / ((1 - x^2) P_n'(x)^2).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double t = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = t; p0 = 1.0; }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
            double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = t; p0 = 1.0; }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
        }
        x[i] = -t;
        x[n - 1 - i] = t;
        double wi = 2.0 / ((1.0 - t * t) * dp * dp);
        w[i] = wi;
        w[n - 1 - i] = wi;
    }
    if (n % 2 == 1) x[n / 2] = 0.0;
}

// Values of the `order` B-splines that are nonzero on the knot span
// [tau[l], tau[l+1]) at z, by the triangular form of the Cox-de Boor recursion
// (eqs. 1-2).  out[r] = B_{l-order+1+r, order}(z).
void nonzero_splines(const std::vector<double>& tau, int l, int order, double z, double* out) {
    double left[8], right[8];
    out[0] = 1.0;
    for (int j = 1; j < order; ++j) {
        left[j] = z - tau[l + 1 - j];
        right[j] = tau[l + j] - z;
        double saved = 0.0;
        for (int r = 0; r < j; ++r) {
            double den = right[r + 1] + left[j - r];
            double tmp = den != 0.0 ? out[r] / den : 0.0;
            out[r] = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        out[j] = saved;
    }
}

void cross_recip(const double* a1, const double* a2, double* b1, double* b2, double* area) {
    double det = a1[0] * a2[1] - a1[1] * a2[0];
    *area = std::fabs(det);
    // b1 . a1 = 2 pi, b1 . a2 = 0, ...
    b1[0] = 2.0 * kPi * a2[1] / det;
    b1[1] = -2.0 * kPi * a2[0] / det;
    b2[0] = -2.0 * kPi * a1[1] / det;
    b2[1] = 2.0 * kPi * a1[0] / det;
}

}  // namespace

bool fft_plan(int n, FftPlan* plan) {
    plan->n = n;
    plan->nr = 0;
    int r = n;
    const int order[4] = {4, 2, 3, 5};
    for (int k = 0; k < 4; ++k) {
        int R = order[k];
        while (r % R == 0) {
            if (plan->nr >= 12) return false;
            plan->rad[plan->nr++] = R;
            r /= R;
        }
    }
    return r == 1;
}

int recommended_ld(int ng) { return (ng + 15) / 16 * 16; }

mb_status build_spline_dir(const std::vector<double>& bp, int K, int nq, SplineDir* out, const char* name) {
    SplineDir& d = *out;
    d.bp = bp;
    d.nint = (int)bp.size() - 1;
    d.nb = d.nint + K - 3;
    d.nq = nq;
    d.nzq = nq * d.nint;
    if (d.nint < 1 || d.nb < 1) return set_error(MB_ERR_INVALID_ARG, "no basis spline left after the hard walls");
    // clamped knot sequence
    std::vector<double> tau;
    for (int j = 0; j < K - 1; ++j) tau.push_back(bp.front());
    for (double v : bp) tau.push_back(v);
    for (int j = 0; j < K - 1; ++j) tau.push_back(bp.back());

    // Gauss rule and spline tables per interval
    std::vector<double> gx, gw;
    gauss_legendre(nq, gx, gw);
    d.zq.resize(d.nzq);
    d.wq.resize(d.nzq);
    d.bval.assign((size_t)d.nzq * K, 0.0);
    d.wbval.assign((size_t)d.nzq * K, 0.0);
    d.dval.assign((size_t)d.nzq * K, 0.0);
    for (int s = 0; s < d.nint; ++s) {
        double a = bp[s], b = bp[s + 1];
        double h = 0.5 * (b - a), mid = 0.5 * (a + b);
        int l = K - 1 + s;
        for (int j = 0; j < nq; ++j) {
            int q = s * nq + j;
            double z = mid + h * gx[j];
            d.zq[q] = z;
            d.wq[q] = h * gw[j];
            double v[8], vl[8];
            nonzero_splines(tau, l, K, z, v);       // full indices s .. s+K-1
            nonzero_splines(tau, l, K - 1, z, vl);  // order K-1: full indices s+1 .. s+K-1
            for (int r = 0; r < K; ++r) {
                int full = s + r;
                int kept = full - 1;
                double val = v[r];
                // derivative, eq. 3
                double dv = 0.0;
                double d1 = tau[full + K - 1] - tau[full];
                double d2 = tau[full + K] - tau[full + 1];
                if (r >= 1 && d1 > 0) dv += (K - 1) / d1 * vl[r - 1];
                if (r <= K - 2 && d2 > 0) dv -= (K - 1) / d2 * vl[r];
                if (kept < 0 || kept >= d.nb) { val = 0.0; dv = 0.0; }
                d.bval[(size_t)q * K + r] = val;
                d.wbval[(size_t)q * K + r] = d.wq[q] * val;
                d.dval[(size_t)q * K + r] = dv;
            }
        }
    }

    // banded overlap and derivative-overlap matrices, band[i][dd] = M[i][i + dd]
    d.sband.assign((size_t)d.nb * K, 0.0);
    d.dband.assign((size_t)d.nb * K, 0.0);
    for (int s = 0; s < d.nint; ++s)
        for (int j = 0; j < nq; ++j) {
            int q = s * nq + j;
            for (int r1 = 0; r1 < K; ++r1)
                for (int r2 = r1; r2 < K; ++r2) {
                    int i = s - 1 + r1, i2 = s - 1 + r2;
                    if (i < 0 || i2 >= d.nb) continue;
                    int dd = r2 - r1;
                    d.sband[(size_t)i * K + dd] += d.wq[q] * d.bval[(size_t)q * K + r1] * d.bval[(size_t)q * K + r2];
                    d.dband[(size_t)i * K + dd] += d.wq[q] * d.dval[(size_t)q * K + r1] * d.dval[(size_t)q * K + r2];
                }
        }

    // banded Cholesky of the overlap, lband[i][dd] = L[i][i - dd]
    d.lband.assign((size_t)d.nb * K, 0.0);
    auto S = [&](int i, int j) -> double {  // symmetric access, |i-j| < K
        if (i > j) std::swap(i, j);
        return d.sband[(size_t)i * K + (j - i)];
    };
    auto L = [&](int i, int j) -> double& { return d.lband[(size_t)i * K + (i - j)]; };
    for (int i = 0; i < d.nb; ++i) {
        int j0 = std::max(0, i - (K - 1));
        for (int j = j0; j <= i; ++j) {
            double sum = S(i, j);
            for (int k = std::max(j0, j - (K - 1)); k < j; ++k) sum -= L(i, k) * L(j, k);
            if (j == i) {
                if (!(sum > 0)) return set_error(MB_ERR_NOT_SPD, std::string(name) + " is not positive definite");
                L(i, i) = std::sqrt(sum);
            } else {
                L(i, j) = sum / L(j, j);
            }
        }
    }
    return MB_OK;
}

mb_status build_tables(const mb_desc* d, Problem* p) {
    if (!d) return set_error(MB_ERR_INVALID_ARG, "desc is NULL");
    if (d->order < 2 || d->order > 6) return set_error(MB_ERR_INVALID_ARG, "order must be 2..6");
    if (d->nbreak < 2 || !d->breakpoints) return set_error(MB_ERR_INVALID_ARG, "need >= 2 breakpoints");
    if (d->nq < 1 || d->nq > 8) return set_error(MB_ERR_INVALID_ARG, "nq must be 1..8");
    if (d->nk < 1 || !d->kfrac) return set_error(MB_ERR_INVALID_ARG, "need >= 1 k-point");
    if (d->natoms < 0 || (d->natoms > 0 && !d->atoms)) return set_error(MB_ERR_INVALID_ARG, "atoms");
    if (d->nspecies < 0 || (d->nspecies > 0 && !d->species)) return set_error(MB_ERR_INVALID_ARG, "species");
    for (int j = 1; j < d->nbreak; ++j)
        if (!(d->breakpoints[j] > d->breakpoints[j - 1]))
            return set_error(MB_ERR_INVALID_ARG, "breakpoints must be strictly increasing");
    p->order = d->order;
    p->nint = d->nbreak - 1;
    p->nb = p->nint + p->order - 3;
    if (p->nb < 1) return set_error(MB_ERR_INVALID_ARG, "no basis spline left after the hard walls");
    p->nq = d->nq;
    p->nzq = p->nq * p->nint;
    p->N1 = d->grid[0];
    p->N2 = d->grid[1];
    if (p->N1 < 2 || p->N2 < 2 || p->N1 > 256 || p->N2 > 256 || !fft_plan(p->N1, &p->plan1) ||
        !fft_plan(p->N2, &p->plan2))
        return set_error(MB_ERR_INVALID_ARG, "grid sizes must be 2..256 with factors 2, 3, 5 only");
    std::memcpy(p->a1, d->a1, sizeof(p->a1));
    std::memcpy(p->a2, d->a2, sizeof(p->a2));
    cross_recip(p->a1, p->a2, p->b1, p->b2, &p->area);
    if (!(p->area > 0)) return set_error(MB_ERR_INVALID_ARG, "degenerate cell");
    p->bp.assign(d->breakpoints, d->breakpoints + d->nbreak);
    p->kfrac.assign(d->kfrac, d->kfrac + 2 * d->nk);
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
    }

    const int K = p->order;
    SplineDir zdir;
    MB_TRY(build_spline_dir(p->bp, K, p->nq, &zdir, "overlap S_z"));
    p->zq = std::move(zdir.zq);
    p->wq = std::move(zdir.wq);
    p->bval = std::move(zdir.bval);
    p->wbval = std::move(zdir.wbval);
    p->sband = std::move(zdir.sband);
    p->dband = std::move(zdir.dband);
    p->lband = std::move(zdir.lband);

    // projectors: z factors (same for every k) and energies
    p->np = 0;
    for (const auto& a : p->atoms)
        if (p->species[a.species].nonlocal) p->np += 4;
    p->Zp.assign((size_t)p->np * p->nb, 0.0);
    p->Ep.assign(p->np, 0.0);
    p->Qp.assign(p->np, 0.0);
    p->zwin.assign((size_t)p->np * 2, 0);
    {
        int pidx = 0;
        for (const auto& a : p->atoms) {
            const mb_species& sp = p->species[a.species];
            if (!sp.nonlocal) continue;
            for (int t = 0; t < 4; ++t, ++pidx) {
                double al = t == 0 ? sp.alpha_s : sp.alpha_p;
                p->Ep[pidx] = t == 0 ? sp.E_s : sp.E_p;
                p->Qp[pidx] = t == 0 ? sp.q_s : sp.q_p;
                if (!std::isfinite(p->Qp[pidx]) || p->Qp[pidx] < 0.0)
                    return set_error(MB_ERR_INVALID_ARG, "augmentation charges q_s, q_p must be finite and >= 0");
                double* Zrow = &p->Zp[(size_t)pidx * p->nb];
                for (int s = 0; s < p->nint; ++s)
                    for (int j = 0; j < p->nq; ++j) {
                        int q = s * p->nq + j;
                        double dz = p->zq[q] - a.pos[2];
                        double f = std::exp(-al * dz * dz);
                        if (t == 3) f *= dz;
                        for (int r = 0; r < K; ++r) {
                            int i = s - 1 + r;
                            if (i < 0 || i >= p->nb) continue;
                            Zrow[i] += p->wbval[(size_t)q * K + r] * f;
                        }
                    }
                double zmax = 0.0;
                for (int i = 0; i < p->nb; ++i) zmax = std::max(zmax, std::fabs(Zrow[i]));
                int lo = p->nb, hi = -1;
                for (int i = 0; i < p->nb; ++i)
                    if (std::fabs(Zrow[i]) > 1e-16 * zmax) { lo = std::min(lo, i); hi = std::max(hi, i); }
                if (hi < 0) { lo = 0; hi = -1; }
                // rows outside the window hold only negligible values: make them exact zeros
                for (int i = 0; i < p->nb; ++i)
                    if (i < lo || i > hi) Zrow[i] = 0.0;
                p->zwin[2 * pidx] = lo;
                p->zwin[2 * pidx + 1] = hi;
            }
        }
    }

    // G sets per k-point
    const int nk = d->nk;
    p->kp.assign(nk, KPoint{});
    for (int ik = 0; ik < nk; ++ik) {
        KPoint& kp = p->kp[ik];
        double f1 = p->kfrac[2 * ik], f2 = p->kfrac[2 * ik + 1];
        double kx = f1 * p->b1[0] + f2 * p->b2[0];
        double ky = f1 * p->b1[1] + f2 * p->b2[1];
        std::vector<std::pair<int, int>> ms;
        if (d->gset_kind == MB_GSET_BOX) {
            if (d->mmax[0] < 0 || d->mmax[1] < 0) return set_error(MB_ERR_INVALID_ARG, "mmax < 0");
            for (int m1 = -d->mmax[0]; m1 <= d->mmax[0]; ++m1)
                for (int m2 = -d->mmax[1]; m2 <= d->mmax[1]; ++m2) ms.emplace_back(m1, m2);
        } else if (d->gset_kind == MB_GSET_SPHERE) {
            if (!(d->ecut > 0)) return set_error(MB_ERR_INVALID_ARG, "ecut must be > 0");
            double r = std::sqrt(2.0 * d->ecut);
            // |m_i| <= |k+G| |a_i| / 2 pi + |f_i|
            int n1 = (int)std::ceil(r * std::hypot(p->a1[0], p->a1[1]) / (2 * kPi)) + 2;
            int n2 = (int)std::ceil(r * std::hypot(p->a2[0], p->a2[1]) / (2 * kPi)) + 2;
            for (int m1 = -n1; m1 <= n1; ++m1)
                for (int m2 = -n2; m2 <= n2; ++m2) {
                    double qx = kx + m1 * p->b1[0] + m2 * p->b2[0];
                    double qy = ky + m1 * p->b1[1] + m2 * p->b2[1];
                    if (0.5 * (qx * qx + qy * qy) <= d->ecut) ms.emplace_back(m1, m2);
                }
        } else {
            return set_error(MB_ERR_INVALID_ARG, "unknown gset_kind");
        }
        if (ms.empty()) return set_error(MB_ERR_INVALID_ARG, "empty G set");
        std::sort(ms.begin(), ms.end());
        kp.ng = (int)ms.size();
        kp.ld = recommended_ld(kp.ng);
        kp.m.resize(2 * kp.ng);
        kp.kg.resize(2 * kp.ng);
        kp.kg2.resize(kp.ng);
        kp.gmap.resize(kp.ng);
        int mmax1 = 0, mmax2 = 0;
        std::vector<char> rowused(p->N1, 0);
        for (int g = 0; g < kp.ng; ++g) {
            int m1 = ms[g].first, m2 = ms[g].second;
            mmax1 = std::max(mmax1, std::abs(m1));
            mmax2 = std::max(mmax2, std::abs(m2));
            kp.m[2 * g] = m1;
            kp.m[2 * g + 1] = m2;
            double qx = kx + m1 * p->b1[0] + m2 * p->b2[0];
            double qy = ky + m1 * p->b1[1] + m2 * p->b2[1];
            kp.kg[2 * g] = qx;
            kp.kg[2 * g + 1] = qy;
            kp.kg2[g] = qx * qx + qy * qy;
            int j1 = ((m1 % p->N1) + p->N1) % p->N1;
            int j2 = ((m2 % p->N2) + p->N2) % p->N2;
            kp.gmap[g] = j1 * p->N2 + j2;
            rowused[j1] = 1;
        }
        if (2 * mmax1 + 1 > p->N1 || 2 * mmax2 + 1 > p->N2)
            return set_error(MB_ERR_INVALID_ARG, "G set does not fit the FFT grid (2 m_max + 1 > N)");
        kp.rows.clear();
        for (int j1 = 0; j1 < p->N1; ++j1)
            if (rowused[j1]) kp.rows.push_back(j1);

        // in-plane projector factors F[p][g] = C e^{-i(k+G).R} Q(k+G) / sqrt(A_c)
        kp.F.assign((size_t)p->np * kp.ld, zd(0.0, 0.0));
        int pidx = 0;
        for (const auto& a : p->atoms) {
            const mb_species& sp = p->species[a.species];
            if (!sp.nonlocal) continue;
            double cs = std::pow(2.0 * sp.alpha_s / kPi, 0.75);
            double cp = std::pow(2.0 * sp.alpha_p / kPi, 0.75) * 2.0 * std::sqrt(sp.alpha_p);
            for (int t = 0; t < 4; ++t, ++pidx) {
                double al = t == 0 ? sp.alpha_s : sp.alpha_p;
                double c = t == 0 ? cs : cp;
                for (int g = 0; g < kp.ng; ++g) {
                    double qx = kp.kg[2 * g], qy = kp.kg[2 * g + 1];
                    double ph = -(qx * a.pos[0] + qy * a.pos[1]);
                    zd phase(std::cos(ph), std::sin(ph));
                    double gauss = (kPi / al) * std::exp(-(qx * qx + qy * qy) / (4.0 * al));
                    zd Q;
                    if (t == 0 || t == 3) Q = zd(gauss, 0.0);
                    else if (t == 1) Q = zd(0.0, -qx / (2.0 * al) * gauss);
                    else Q = zd(0.0, -qy / (2.0 * al) * gauss);
                    kp.F[(size_t)pidx * kp.ld + g] = c * phase * Q / std::sqrt(p->area);
                }
            }
        }
    }
    return build_augmentation(p);
}

// Ultrasoft overlap S = S_0 + B Q B^H (S_0 = I_G (x) S_z, columns of B the projectors
// beta_p = F_p (x) Z_p, Q = diag(q_p); Sec. II.B.2).  The Woodbury identity
//   S^{-1} = S_0^{-1} - S_0^{-1} B W B^H S_0^{-1},  W = Q (I + C Q)^{-1},  C = B^H S_0^{-1} B,
// needs only the N_p x N_p matrix W per k-point: C[a][b] = (sum_G conj(F_a(G)) F_b(G)) *
// (sum_i Z_a(i) (S_z^{-1} Z_b)(i)), since S_0^{-1} acts on the z factor alone.  I + C Q is
// inverted by Gauss-Jordan elimination with partial pivoting (it is nonsingular: C is
// positive semidefinite and Q >= 0, so C Q has no negative eigenvalue).
mb_status build_augmentation(Problem* p) {
    p->uspp = false;
    for (double q : p->Qp)
        if (q != 0.0) p->uspp = true;
    for (auto& kp : p->kp) kp.W.clear();
    if (!p->uspp) return MB_OK;
    const int np = p->np, nb = p->nb, K = p->order;
    // Z'_b = S_z^{-1} Z_b by forward and back substitution with lband[i][d] = L[i][i-d]
    std::vector<double> Zs(p->Zp);
    for (int b = 0; b < np; ++b) {
        double* x = &Zs[(size_t)b * nb];
        for (int i = 0; i < nb; ++i) {
            double v = x[i];
            for (int d = 1; d < K && d <= i; ++d) v -= p->lband[(size_t)i * K + d] * x[i - d];
            x[i] = v / p->lband[(size_t)i * K];
        }
        for (int i = nb - 1; i >= 0; --i) {
            double v = x[i];
            for (int d = 1; d < K && i + d < nb; ++d) v -= p->lband[(size_t)(i + d) * K + d] * x[i + d];
            x[i] = v / p->lband[(size_t)i * K];
        }
    }
    std::vector<double> Cz((size_t)np * np, 0.0);
    for (int a = 0; a < np; ++a)
        for (int b = 0; b < np; ++b) {
            double acc = 0.0;
            for (int i = 0; i < nb; ++i) acc += p->Zp[(size_t)a * nb + i] * Zs[(size_t)b * nb + i];
            Cz[(size_t)a * np + b] = acc;
        }
    std::vector<zd> A((size_t)np * np), Ai((size_t)np * np);
    for (auto& kp : p->kp) {
        for (int a = 0; a < np; ++a)
            for (int b = 0; b < np; ++b) {
                zd cf(0.0, 0.0);
                const zd* Fa = &kp.F[(size_t)a * kp.ld];
                const zd* Fb = &kp.F[(size_t)b * kp.ld];
                for (int g = 0; g < kp.ng; ++g) cf += std::conj(Fa[g]) * Fb[g];
                A[(size_t)a * np + b] = (a == b ? zd(1.0, 0.0) : zd(0.0, 0.0)) + cf * Cz[(size_t)a * np + b] * p->Qp[b];
                Ai[(size_t)a * np + b] = a == b ? zd(1.0, 0.0) : zd(0.0, 0.0);
            }
        for (int col = 0; col < np; ++col) {
            int piv = col;
            for (int r = col + 1; r < np; ++r)
                if (std::abs(A[(size_t)r * np + col]) > std::abs(A[(size_t)piv * np + col])) piv = r;
            if (!(std::abs(A[(size_t)piv * np + col]) > 0.0))
                return set_error(MB_ERR_NOT_SPD, "ultrasoft overlap: I + C Q is singular");
            if (piv != col)
                for (int j = 0; j < np; ++j) {
                    std::swap(A[(size_t)piv * np + j], A[(size_t)col * np + j]);
                    std::swap(Ai[(size_t)piv * np + j], Ai[(size_t)col * np + j]);
                }
            const zd inv = 1.0 / A[(size_t)col * np + col];
            for (int j = 0; j < np; ++j) {
                A[(size_t)col * np + j] *= inv;
                Ai[(size_t)col * np + j] *= inv;
            }
            for (int r = 0; r < np; ++r) {
                if (r == col) continue;
                const zd f = A[(size_t)r * np + col];
                if (f == zd(0.0, 0.0)) continue;
                for (int j = 0; j < np; ++j) {
                    A[(size_t)r * np + j] -= f * A[(size_t)col * np + j];
                    Ai[(size_t)r * np + j] -= f * Ai[(size_t)col * np + j];
                }
            }
        }
        kp.W.assign((size_t)np * np, zd(0.0, 0.0));
        for (int a = 0; a < np; ++a)
            for (int b = 0; b < np; ++b) kp.W[(size_t)a * np + b] = p->Qp[a] * Ai[(size_t)a * np + b];
    }
    return MB_OK;
}

}  // namespace mb
