// Host side of the molecule load: validation, normalisation constants and
// the integer layout tables of rows, component pairs and terms.  The pair
// arithmetic itself runs on the device (prep.hip).
//
// Normalisation (App. A, eq. defprimitive and N_alpha): every primitive is
// scaled to unit self-overlap, written per axis with the Gaussian moment
// int x^{2i} e^{-2 alpha x^2} dx = (2i-1)!!/(4 alpha)^i sqrt(pi/(2 alpha));
// with normalise = 1 every contracted Cartesian component is then scaled to
// unit norm.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <climits>
#include <cstdint>

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


// Norm factor of x^i exp(-alpha x^2) on one axis: [int x^{2i} e^{-2 alpha x^2} dx]^{-1/2}.
// App. A's N_alpha is the product of these over the three axes.
double norm1d(double alpha, int i) {
    return 1.0 / std::sqrt(dfact(2 * i - 1) / std::pow(4.0 * alpha, i) * std::sqrt(M_PI / (2.0 * alpha)));
}


}  // namespace

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
    std::vector<int> bf_shell, bf_pw;   // shell and Cartesian powers of each AO
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
            bf_shell.push_back(s);
            for (int a = 0; a < 3; ++a) bf_pw.push_back(kCart[shell_l[s]][c][a]);
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
    // 1D normalisation factors per primitive for powers 0..2
    nb.n1d.resize(nb.exps.size() * 3);
    for (size_t k = 0; k < nb.exps.size(); ++k)
        for (int i = 0; i < 3; ++i) nb.n1d[3 * k + i] = norm1d(nb.exps[k], i);
    nb.cnorm.assign(bf, 1.0);
    if (nb.normalise) {
        // <chi_k|chi_l> of two normalised primitives of one shell, per axis
        // n_k(i) n_l(i) (2i-1)!! / (2p)^i sqrt(pi/p) with p = a_k + a_l; the
        // primitive factors come from n1d, (2i-1)!! = 1, 1, 3 for i = 0, 1, 2
        const double df[3] = {1.0, 1.0, 3.0};
        for (int mu = 0; mu < bf; ++mu) {
            const int s = bf_shell[mu];
            const int* pw = &bf_pw[3 * mu];
            const int o = nb.sh_off[s], np = nb.sh_nprim[s];
            double sum = 0.0;
            for (int k = 0; k < np; ++k)
                for (int l = 0; l < np; ++l) {
                    const double p = nb.exps[o + k] + nb.exps[o + l];
                    const double sq = std::sqrt(M_PI / p), tp = 2.0 * p;
                    double t = sq * sq * sq;
                    for (int ax = 0; ax < 3; ++ax) {
                        const int i = pw[ax];
                        t *= nb.n1d[3 * (o + k) + i] * nb.n1d[3 * (o + l) + i] * df[i] /
                             (i == 0 ? 1.0 : i == 1 ? tp : tp * tp);
                    }
                    sum += nb.coefs[o + k] * nb.coefs[o + l] * t;
                }
            if (!(sum > 0.0)) return "contracted function with zero norm";
            nb.cnorm[mu] = 1.0 / std::sqrt(sum);
        }
    }
    // layout of rows (primitive pair x axis x power pair), component pairs
    // (mu <= nu) and terms (component pair x primitive pair), per shell pair
    for (int s = 0; s < n_shells; ++s) nb.shells.push_back(PrepShell{nb.sh_atom[s], nb.sh_l[s], nb.sh_nprim[s], nb.sh_off[s]});
    {
        // sizes first, so the tables are filled without reallocation
        long long ncp_all = 0;
        for (int sA = 0; sA < n_shells; ++sA)
            for (int sB = sA; sB < n_shells; ++sB) {
                const int lA = nb.sh_l[sA], lB = nb.sh_l[sB];
                ncp_all += sA == sB ? ncart(lA) * (ncart(lA) + 1) / 2 : ncart(lA) * ncart(lB);
            }
        const size_t nsp = (size_t)n_shells * (n_shells + 1) / 2;
        if (ncp_all > INT32_MAX / 2) return "molecule too large for 32-bit term indexing";
        nb.sp.reserve(4 * nsp);
        nb.sp_cp.reserve(nsp);
        nb.cp_first.reserve((size_t)ncp_all);
        nb.cp_nterms.reserve((size_t)ncp_all);
    }
    long long rows = 0, terms = 0;
    long long cps = 0;
    for (int sA = 0; sA < n_shells; ++sA)
        for (int sB = sA; sB < n_shells; ++sB) {
            const int lA = nb.sh_l[sA], lB = nb.sh_l[sB];
            const int npp = nb.sh_nprim[sA] * nb.sh_nprim[sB];
            const int ncp = sA == sB ? ncart(lA) * (ncart(lA) + 1) / 2 : ncart(lA) * ncart(lB);
            if (rows > INT32_MAX / 2 || terms > INT32_MAX / 2 || cps > INT32_MAX / 2)
                return "molecule too large for 32-bit term indexing";
            nb.sp.push_back(sA);
            nb.sp.push_back(sB);
            nb.sp.push_back((int)rows);
            nb.sp.push_back((int)terms);
            nb.sp_cp.push_back((int)cps);
            for (int c = 0; c < ncp; ++c) {
                nb.cp_first.push_back((int)(terms + (long long)c * npp));
                nb.cp_nterms.push_back(npp);
            }
            rows += (long long)npp * 3 * (lA + 1) * (lB + 1);
            terms += (long long)ncp * npp;
            cps += ncp;
        }
    nb.n_sp = (int)nb.sp_cp.size();
    nb.n_cp = (int)cps;
    nb.n_rows = rows;
    nb.n_terms = terms;
    b = std::move(nb);
    return "";
}

}  // namespace scff
