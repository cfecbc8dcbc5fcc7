// Host precompute of the Cartesian form-factor engine (FP64).
//
// Paper Sec. 5.3: the small q-independent pair coefficients (eqs. Mij,
// sigmaTidbits, positionTidbits, bCoefficients) are computed once per
// molecule; Sec. 4 eq. Ccoefficients gives the monomial form of each 1D
// polynomial that the device evaluates.  Sec. 5.3 also describes the
// per-transition thresholding of pair terms, implemented here with a
// q-independent magnitude bound so that the dropped part is controlled.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "engine.h"

namespace scff {

namespace {

const int kCart[3][6][3] = {
    {{0, 0, 0}},
    {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}},
    {{2, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}},
};

int ncart(int l) { return (l + 1) * (l + 2) / 2; }

double dfact(int n) {  // n!!, (-1)!! = 1
    double r = 1.0;
    for (int k = n; k > 1; k -= 2) r *= k;
    return r;
}

double fact(int n) {
    double r = 1.0;
    for (int k = 2; k <= n; ++k) r *= k;
    return r;
}

double choose(int n, int k) {
    if (k < 0 || k > n) return 0.0;
    return fact(n) / (fact(k) * fact(n - k));
}

// Norm factor of x^i exp(-alpha x^2) on one axis: [int x^{2i} e^{-2 alpha x^2} dx]^{-1/2}.
// App. A's N_alpha is the product of these over the three axes.
double norm1d(double alpha, int i) {
    return 1.0 / std::sqrt(dfact(2 * i - 1) / std::pow(4.0 * alpha, i) * std::sqrt(M_PI / (2.0 * alpha)));
}

// max_q |q|^u exp(-q^2/(4p)) = (2 p u / e)^{u/2}; 1 for u = 0.
double moment_peak(double p, int u) {
    if (u == 0) return 1.0;
    return std::pow(2.0 * p * u / M_E, 0.5 * u);
}

}  // namespace

uint16_t bf16_rne(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf/nan passthrough
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

float bf16_to_float(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float x;
    std::memcpy(&x, &u, 4);
    return x;
}

std::string build_basis(Basis& b, int n_atoms, const double* xyz, int n_shells,
                        const int* shell_atom, const int* shell_l, const int* shell_nprim,
                        const double* exps, const double* coefs, int normalise) {
    if (n_atoms <= 0 || n_shells <= 0) return "n_atoms and n_shells must be positive";
    if (!xyz || !shell_atom || !shell_l || !shell_nprim || !exps || !coefs)
        return "NULL input array";
    Basis nb;
    nb.n_atoms = n_atoms;
    nb.n_shells = n_shells;
    nb.normalise = normalise != 0;
    nb.xyz.assign(xyz, xyz + 3 * n_atoms);
    for (double v : nb.xyz)
        if (!std::isfinite(v)) return "non-finite atom coordinate";
    int off = 0, bf = 0;
    for (int s = 0; s < n_shells; ++s) {
        if (shell_atom[s] < 0 || shell_atom[s] >= n_atoms) return "shell_atom out of range";
        if (shell_l[s] < 0 || shell_l[s] > 2) return "shell_l must be 0, 1 or 2";
        if (shell_nprim[s] < 1 || shell_nprim[s] > kMaxPrim) return "shell_nprim must be in 1..32";
        nb.sh_atom.push_back(shell_atom[s]);
        nb.sh_l.push_back(shell_l[s]);
        nb.sh_nprim.push_back(shell_nprim[s]);
        nb.sh_off.push_back(off);
        nb.sh_bf0.push_back(bf);
        for (int c = 0; c < ncart(shell_l[s]); ++c) {
            nb.bf_shell.push_back(s);
            for (int a = 0; a < 3; ++a) nb.bf_pw.push_back(kCart[shell_l[s]][c][a]);
        }
        off += shell_nprim[s];
        bf += ncart(shell_l[s]);
    }
    nb.nbf = bf;
    nb.exps.assign(exps, exps + off);
    nb.coefs.assign(coefs, coefs + off);
    for (int k = 0; k < off; ++k) {
        if (!(exps[k] > 0.0) || !std::isfinite(exps[k])) return "exponents must be positive and finite";
        if (!std::isfinite(coefs[k])) return "non-finite contraction coefficient";
    }
    nb.cnorm.assign(bf, 1.0);
    if (nb.normalise) {
        for (int mu = 0; mu < bf; ++mu) {
            int s = nb.bf_shell[mu];
            const int* pw = &nb.bf_pw[3 * mu];
            double sum = 0.0;
            for (int k = 0; k < nb.sh_nprim[s]; ++k)
                for (int l = 0; l < nb.sh_nprim[s]; ++l) {
                    double a = nb.exps[nb.sh_off[s] + k], c = nb.exps[nb.sh_off[s] + l];
                    double p = a + c, t = 1.0;
                    for (int ax = 0; ax < 3; ++ax)
                        t *= norm1d(a, pw[ax]) * norm1d(c, pw[ax]) * dfact(2 * pw[ax] - 1) /
                             std::pow(2.0 * p, pw[ax]) * std::sqrt(M_PI / p);
                    sum += nb.coefs[nb.sh_off[s] + k] * nb.coefs[nb.sh_off[s] + l] * t;
                }
            if (!(sum > 0.0)) return "contracted function with zero norm";
            nb.cnorm[mu] = 1.0 / std::sqrt(sum);
        }
    }
    b = std::move(nb);
    return "";
}

void build_pairs(const Basis& b, PairData& pd) {
    pd = PairData();
    for (int sA = 0; sA < b.n_shells; ++sA)
        for (int sB = sA; sB < b.n_shells; ++sB) {
            ++pd.shell_pairs;
            const int lA = b.sh_l[sA], lB = b.sh_l[sB];
            const double* A = &b.xyz[3 * b.sh_atom[sA]];
            const double* B = &b.xyz[3 * b.sh_atom[sB]];
            const int ncls = (lA + 1) * (lB + 1);
            double AB2 = 0.0;
            for (int a = 0; a < 3; ++a) AB2 += (A[a] - B[a]) * (A[a] - B[a]);
            const int npa = b.sh_nprim[sA], npb = b.sh_nprim[sB];
            std::vector<int> rowbase(npa * npb);
            std::vector<double> pp_p(npa * npb);
            for (int k = 0; k < npa; ++k)
                for (int l = 0; l < npb; ++l) {
                    const double al = b.exps[b.sh_off[sA] + k], be = b.exps[b.sh_off[sB] + l];
                    const double p = al + be;
                    // Gaussian product prefactor and contraction coefficients (eq. Mij with
                    // sigma^2 = 1/(2 alpha); (2 pi)^{3/2} sigma_ij^3 = (pi/p)^{3/2}).
                    const double pref = b.coefs[b.sh_off[sA] + k] * b.coefs[b.sh_off[sB] + l] *
                                         std::pow(M_PI / p, 1.5) * std::exp(-al * be / p * AB2);
                    rowbase[k * npb + l] = (int)pd.rows.size();
                    pp_p[k * npb + l] = p;
                    for (int ax = 0; ax < 3; ++ax) {
                        const double P = (al * A[ax] + be * B[ax]) / p;  // eq. positionTidbits
                        const double PA = P - A[ax], PB = P - B[ax];
                        for (int i = 0; i <= lA; ++i)
                            for (int j = 0; j <= lB; ++j) {
                                // b_t: coefficients of y^t in (y + PA)^i (y + PB)^j (eq. bCoefficients)
                                double bt[5] = {0, 0, 0, 0, 0};
                                for (int k1 = 0; k1 <= i; ++k1)
                                    for (int k2 = 0; k2 <= j; ++k2)
                                        bt[k1 + k2] += choose(i, k1) * choose(j, k2) *
                                                       std::pow(PA, i - k1) * std::pow(PB, j - k2);
                                // e_u of eq. Ccoefficients with sigma_ij^2 = 1/(2p), divided by i^u
                                VRow r{};
                                r.p = p;
                                r.P = P;
                                r.axis = ax;
                                r.deg = i + j;
                                const double scale =
                                    norm1d(al, i) * norm1d(be, j) * (ax == 0 ? pref : 1.0);
                                for (int u = 0; u <= i + j; ++u) {
                                    double s = 0.0;
                                    for (int m = 0; u + 2 * m <= i + j; ++m)
                                        s += bt[u + 2 * m] * fact(u + 2 * m) /
                                             (fact(m) * fact(u) * std::pow(2.0, m)) /
                                             std::pow(2.0 * p, u + m);
                                    r.e[u] = s * scale;
                                }
                                pd.rows.push_back(r);
                            }
                    }
                }
            // component pairs mu <= nu of this shell pair and their terms
            for (int c1 = 0; c1 < ncart(lA); ++c1)
                for (int c2 = (sA == sB ? c1 : 0); c2 < ncart(lB); ++c2) {
                    CompPair cp;
                    cp.mu = b.sh_bf0[sA] + c1;
                    cp.nu = b.sh_bf0[sB] + c2;
                    cp.first_term = (int)pd.terms.size();
                    cp.n_terms = npa * npb;
                    const int* pa = kCart[lA][c1];
                    const int* pb = kCart[lB][c2];
                    for (int pp = 0; pp < npa * npb; ++pp) {
                        Term t;
                        double bound = 1.0;
                        for (int ax = 0; ax < 3; ++ax) {
                            t.row[ax] = rowbase[pp] + ax * ncls + pa[ax] * (lB + 1) + pb[ax];
                            const VRow& r = pd.rows[t.row[ax]];
                            double s = 0.0;
                            for (int u = 0; u <= r.deg; ++u)
                                s += std::fabs(r.e[u]) * moment_peak(pp_p[pp], u);
                            bound *= s;
                        }
                        t.bound = bound;
                        pd.terms.push_back(t);
                    }
                    pd.prim_pairs_total += npa * npb;
                    pd.cps.push_back(cp);
                }
        }
}

std::string pack(const Basis& b, const PairData& pd, int n_states, const double* T,
                 double screen_eps, double spin_factor, Packed& out) {
    if (n_states < 1 || n_states > kMaxStates) return "n_states must be in 1..32";
    const int nbf = b.nbf;
    const int ncp = (int)pd.cps.size();
    Packed pk;
    pk.n_states = n_states;
    pk.state_blocks = (n_states + kStateBlock - 1) / kStateBlock;
    pk.pairs_total = ncp;
    const int SW = kStateBlock * pk.state_blocks;

    // Tp(s, k) = (T_mn + T_nm or T_mm) * c_m c_n * s_f   (i <-> j symmetry of Omega)
    std::vector<double> tp((size_t)ncp * n_states);
    for (int k = 0; k < ncp; ++k) {
        const int m = pd.cps[k].mu, n = pd.cps[k].nu;
        const double cc = b.cnorm[m] * b.cnorm[n] * spin_factor;
        for (int s = 0; s < n_states; ++s) {
            const double* Ts = T + (size_t)s * nbf * nbf;
            double v = (m == n) ? Ts[(size_t)m * nbf + m]
                                : Ts[(size_t)m * nbf + n] + Ts[(size_t)n * nbf + m];
            if (!std::isfinite(v)) return "non-finite entry in T";
            tp[(size_t)k * n_states + s] = v * cc;
        }
    }

    // Screening: drop the terms of smallest weight while, for every state, the
    // summed bounds of dropped terms stay <= eps * (sum of all term bounds).
    const size_t nt = pd.terms.size();
    std::vector<char> keep(nt, 1);
    std::vector<int> term_cp(nt);
    for (int k = 0; k < ncp; ++k)
        for (int t = 0; t < pd.cps[k].n_terms; ++t) term_cp[pd.cps[k].first_term + t] = k;
    if (screen_eps > 0.0) {
        std::vector<double> tot(n_states, 0.0);
        for (size_t t = 0; t < nt; ++t)
            for (int s = 0; s < n_states; ++s)
                tot[s] += std::fabs(tp[(size_t)term_cp[t] * n_states + s]) * pd.terms[t].bound;
        std::vector<double> w(nt, 0.0);
        for (size_t t = 0; t < nt; ++t)
            for (int s = 0; s < n_states; ++s)
                if (tot[s] > 0.0)
                    w[t] = std::max(w[t], std::fabs(tp[(size_t)term_cp[t] * n_states + s]) *
                                              pd.terms[t].bound / tot[s]);
        std::vector<size_t> order(nt);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return w[x] < w[y]; });
        double cum = 0.0;
        for (size_t i = 0; i < nt; ++i) {
            const size_t t = order[i];
            if (cum + w[t] > screen_eps) break;
            cum += w[t];
            keep[t] = 0;
        }
    }

    // virtual pairs of <= kMaxTermsPerPair kept terms each
    struct VP { int cp; std::vector<int> terms; };
    std::vector<VP> vps;
    long long kept_pairs = 0, kept_terms = 0;
    for (int k = 0; k < ncp; ++k) {
        std::vector<int> kt;
        for (int t = 0; t < pd.cps[k].n_terms; ++t)
            if (keep[pd.cps[k].first_term + t]) kt.push_back(pd.cps[k].first_term + t);
        if (kt.empty()) continue;
        ++kept_pairs;
        kept_terms += (long long)kt.size();
        const int nv = ((int)kt.size() + kMaxTermsPerPair - 1) / kMaxTermsPerPair;
        size_t pos = 0;
        for (int v = 0; v < nv; ++v) {
            const size_t take = (kt.size() - pos) / (size_t)(nv - v);
            VP vp;
            vp.cp = k;
            vp.terms.assign(kt.begin() + pos, kt.begin() + pos + take);
            pos += take;
            vps.push_back(std::move(vp));
        }
    }
    std::stable_sort(vps.begin(), vps.end(),
                     [](const VP& x, const VP& y) { return x.terms.size() > y.terms.size(); });
    if (vps.empty()) {  // everything screened away (or T == 0): one empty chunk
        VP vp;
        vp.cp = -1;
        vps.push_back(vp);
    }
    while (vps.size() % kChunk) vps.push_back(VP{-1, {}});
    pk.n_vpairs = (int)vps.size();
    pk.n_chunks = pk.n_vpairs / kChunk;
    pk.pairs_kept = kept_pairs;
    pk.terms_kept = kept_terms;

    // compact the rows referenced by kept terms; row 0 is all zero and is
    // what padded terms (beyond a pair's own terms) point to
    {
        VRowDev z{};
        z.inv4p = 1.0;
        pk.rows.push_back(z);
    }
    std::vector<int> remap(pd.rows.size(), -1);
    auto row_id = [&](int r) {
        if (remap[r] < 0) {
            remap[r] = (int)pk.rows.size();
            const VRow& v = pd.rows[r];
            VRowDev d{};
            d.P = v.P;
            d.inv4p = 0.25 / v.p;
            for (int u = 0; u < 5; ++u) d.e[u] = (u <= v.deg) ? v.e[u] : 0.0;
            d.deg = v.deg;
            d.axis = v.axis;
            pk.rows.push_back(d);
        }
        return remap[r];
    };

    pk.tp.assign((size_t)pk.n_vpairs * SW, 0.0f);
    for (int c = 0; c < pk.n_chunks; ++c) {
        int npp = 1;
        for (int j = 0; j < kChunk; ++j) npp = std::max(npp, (int)vps[c * kChunk + j].terms.size());
        pk.chunk_off.push_back((int)(pk.terms.size() / 4));
        pk.chunk_npp.push_back(npp);
        for (int j = 0; j < kChunk; ++j) {
            const VP& vp = vps[c * kChunk + j];
            for (int q = 0; q < npp; ++q) {
                if (q < (int)vp.terms.size()) {
                    const Term& t = pd.terms[vp.terms[q]];
                    pk.terms.push_back(row_id(t.row[0]));
                    pk.terms.push_back(row_id(t.row[1]));
                    pk.terms.push_back(row_id(t.row[2]));
                    pk.terms.push_back(1);
                } else {
                    for (int z = 0; z < 3; ++z) pk.terms.push_back(0);
                    pk.terms.push_back(0);
                }
            }
            if (vp.cp >= 0)
                for (int s = 0; s < n_states; ++s)
                    pk.tp[(size_t)(c * kChunk + j) * SW + s] = (float)tp[(size_t)vp.cp * n_states + s];
        }
    }
    pk.tp_hi.resize(pk.tp.size());
    pk.tp_lo.resize(pk.tp.size());
    for (size_t i = 0; i < pk.tp.size(); ++i) {
        const uint16_t h = bf16_rne(pk.tp[i]);
        pk.tp_hi[i] = h;
        pk.tp_lo[i] = bf16_rne(pk.tp[i] - bf16_to_float(h));
    }
    out = std::move(pk);
    return "";
}

}  // namespace scff
