// Host tables of the spherical method (paper Sec. 4 eqs. WTensor, YYY,
// RTensor; App. B), FP64, independent of the molecule:
//
//   Theta[uvw][nlm]   the monomial-to-harmonic coefficients of App. B,
//                     q_x^u q_y^v q_z^w = |q|^n sum_{lam,mu} Theta Y_lam^mu(q^),
//                     n = u + v + w <= 4;
//   Gaunt[lm][lm'][j] the coupling of eq. YYY,
//                     Y_lam^mu Y_L^M = sum_{l,m} G Y_l^m (m = mu + M),
//                     for lam <= 4, l <= lmax and L = |l - lam| + 2 j.
//
// Both are integrals of products of spherical harmonics over the unit sphere
// and are computed here with a product rule (Gauss-Legendre nodes in
// cos theta, equally spaced azimuths) that integrates every such product of
// the degrees involved exactly; by orthonormality that equals App. B's
// recursion and the Wigner-3j form of the Gaunt coefficients.
#include <array>
#include <cmath>
#include <complex>
#include <vector>

#include "engine.h"

namespace scff {

namespace {

using cd = std::complex<double>;

// Complex Y_l^m (Condon-Shortley phase, orthonormal) for l <= lmax at one
// direction, index l^2 + l + m; associated Legendre functions by upward
// recurrence in l from the normalised P_m^m.
void ylm_row(int lmax, double theta, double phi, cd* out) {
    const double x = std::cos(theta), sx = std::sin(theta);
    double pmm = std::sqrt(1.0 / (4.0 * M_PI));
    for (int m = 0; m <= lmax; ++m) {
        if (m > 0) pmm *= -std::sqrt((2.0 * m + 1.0) / (2.0 * m)) * sx;
        const cd e = std::polar(1.0, m * phi);
        double p2 = 0.0, p1 = pmm;
        for (int l = m; l <= lmax; ++l) {
            double cur;
            if (l == m) {
                cur = pmm;
            } else if (l == m + 1) {
                cur = std::sqrt(2.0 * m + 3.0) * x * pmm;
            } else {
                const double a = std::sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
                const double b = std::sqrt(((l - 1.0) * (l - 1.0) - (double)m * m) / (4.0 * (l - 1.0) * (l - 1.0) - 1.0));
                cur = a * (x * p1 - b * p2);
            }
            if (l > m) {
                p2 = p1;
                p1 = cur;
            }
            const cd y = cur * e;
            out[l * l + l + m] = y;
            if (m > 0) out[l * l + l - m] = ((m & 1) ? -1.0 : 1.0) * std::conj(y);
        }
    }
}

void gauss_legendre_nodes(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

struct Rule {
    std::vector<double> theta, phi, w;
};

// exact for products of harmonics of total degree < 2 nt
Rule sphere_rule(int nt) {
    Rule r;
    std::vector<double> x, w;
    gauss_legendre_nodes(nt, x, w);
    const int np = 2 * nt + 1;
    for (int i = 0; i < nt; ++i)
        for (int j = 0; j < np; ++j) {
            r.theta.push_back(std::acos(x[i]));
            r.phi.push_back(2.0 * M_PI * j / np);
            r.w.push_back(w[i] * 2.0 * M_PI / np);
        }
    return r;
}

}  // namespace

SphIndex sph_index() {
    SphIndex ix;
    for (int n = 0; n <= kSphMaxN; ++n)
        for (int lam = n; lam >= 0; lam -= 2)
            for (int mu = -lam; mu <= lam; ++mu) ix.nlm.push_back({n, lam, mu});
    for (int u = 0; u <= kSphMaxN; ++u)
        for (int v = 0; u + v <= kSphMaxN; ++v)
            for (int w = 0; u + v + w <= kSphMaxN; ++w) ix.uvw.push_back({u, v, w});
    return ix;
}

std::vector<double> sph_theta_table(const SphIndex& ix) {
    // Theta^{uvw}_{lam mu} = int x^u y^v z^w Y_lam^mu* dOmega (degree <= 8: nt = 6 is exact)
    const Rule r = sphere_rule(6);
    const int nl = (kSphMaxN + 1) * (kSphMaxN + 1);
    std::vector<cd> Y(nl);
    const size_t nu = ix.uvw.size(), nn = ix.nlm.size();
    std::vector<cd> th(nu * nn, cd(0.0, 0.0));
    for (size_t k = 0; k < r.w.size(); ++k) {
        ylm_row(kSphMaxN, r.theta[k], r.phi[k], Y.data());
        const double sx = std::sin(r.theta[k]);
        const double d[3] = {sx * std::cos(r.phi[k]), sx * std::sin(r.phi[k]), std::cos(r.theta[k])};
        for (size_t a = 0; a < nu; ++a) {
            const auto& p = ix.uvw[a];
            const double mono = std::pow(d[0], p[0]) * std::pow(d[1], p[1]) * std::pow(d[2], p[2]);
            const int n = p[0] + p[1] + p[2];
            for (size_t b = 0; b < nn; ++b) {
                const auto& q = ix.nlm[b];
                if (q[0] != n) continue;
                th[a * nn + b] += r.w[k] * mono * std::conj(Y[q[1] * q[1] + q[1] + q[2]]);
            }
        }
    }
    std::vector<double> out(2 * nu * nn);
    for (size_t i = 0; i < nu * nn; ++i) {
        // exact zeros stay zero: entries below rounding of the rule are cleared
        out[2 * i] = std::fabs(th[i].real()) < 1e-14 ? 0.0 : th[i].real();
        out[2 * i + 1] = std::fabs(th[i].imag()) < 1e-14 ? 0.0 : th[i].imag();
    }
    return out;
}

std::vector<double> sph_gaunt_table(int lmax) {
    // G[lm'][lm][j] = int Y_lam^mu Y_L^M Y_l^m* dOmega with L = |l - lam| + 2 j,
    // M = m - mu; real.  Degrees up to kSphMaxN + (lmax + kSphMaxN) + lmax.
    const int Lmax = lmax + kSphMaxN;
    const int nt = (kSphMaxN + Lmax + lmax) / 2 + 1;
    const Rule r = sphere_rule(nt);
    const int nL = (Lmax + 1) * (Lmax + 1), nl = (lmax + 1) * (lmax + 1), nlam = (kSphMaxN + 1) * (kSphMaxN + 1);
    std::vector<double> G((size_t)nlam * nl * kSphGauntJ, 0.0);
    std::vector<cd> Y(nL);
    for (size_t k = 0; k < r.w.size(); ++k) {
        ylm_row(Lmax, r.theta[k], r.phi[k], Y.data());
        for (int lam = 0; lam <= kSphMaxN; ++lam)
            for (int mu = -lam; mu <= lam; ++mu) {
                const cd a = r.w[k] * Y[lam * lam + lam + mu];
                for (int l = 0; l <= lmax; ++l)
                    for (int m = -l; m <= l; ++m) {
                        const cd b = a * std::conj(Y[l * l + l + m]);
                        const int M = m - mu;
                        for (int j = 0; j < kSphGauntJ; ++j) {
                            const int L = std::abs(l - lam) + 2 * j;
                            if (L > l + lam || std::abs(M) > L) continue;
                            G[((size_t)(lam * lam + lam + mu) * nl + (l * l + l + m)) * kSphGauntJ + j] +=
                                (b * Y[L * L + L + M]).real();
                        }
                    }
            }
    }
    return G;
}

}  // namespace scff
