/*
 * FP64 CPU oracle for the molecular transition form factor
 *
 *     f_s(q) = s_f * sum_{mu,nu} T^s_{mu nu} * Omega_{mu nu}(q),
 *     Omega_{mu nu}(q) = integral d^3r  phi_mu(r) phi_nu(r) exp(+i q.r),
 *
 * i.e. the AO-basis form of the form factor (paper Sec. 4, first equation;
 * Sec. 2.2 / eq. fSreal and eq. PhiTDM for the definition, with the
 * spin-degeneracy factor sqrt(2) of Sec. 2.2 made the caller's choice s_f).
 *
 * TEST INFRASTRUCTURE.  This file is the checker, not the product: only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg load it.
 * It shares no code, header, table or helper with the HIP library.
 *
 * What it computes, step by step (all FP64, no screening, no symmetry
 * packing, full double sum over component pairs and primitive pairs):
 *
 *  1. Components.  A shell (atom A, angular momentum l, primitives
 *     {alpha_k, d_k}) expands to Cartesian monomials x^a y^b z^c with
 *     a+b+c = l, in the order s; x,y,z; xx,xy,xz,yy,yz,zz (App. A,
 *     eq. defprimitive, with every Cartesian prefactor k_i = 1).
 *  2. Primitive normalisation n_k: each primitive x^a y^b z^c e^{-alpha r^2}
 *     is scaled to unit self-overlap.  This is App. A's N_alpha written with
 *     sigma^2 = 1/(2 alpha) and the Gaussian moment
 *     int x^{2a} e^{-2 alpha x^2} dx = (2a-1)!!/(4 alpha)^a sqrt(pi/(2 alpha)).
 *  3. Contracted normalisation (normalise = 1): every contracted Cartesian
 *     component is rescaled to unit self-overlap, c_mu = S_mumu^{-1/2}.
 *     With normalise = 0 the coefficients d_k n_k are taken as given.
 *  4. For one primitive pair (alpha on A, beta on B) and one axis with powers
 *     (i, j) the 1D integral
 *         I(q) = int (x-A)^i (x-B)^j e^{-alpha (x-A)^2 - beta (x-B)^2} e^{i q x} dx
 *     is evaluated in closed form: the Gaussian product theorem
 *     (p = alpha+beta, P = (alpha A + beta B)/p) gives
 *     e^{-alpha beta (A-B)^2/p} e^{-p (x-P)^2}; completing the square with
 *     the plane wave shifts the centre to P + i q/(2p), and the binomial
 *     expansion in the shifted variable leaves even Gaussian moments:
 *         I(q) = sqrt(pi/p) e^{-alpha beta (A-B)^2/p} e^{-q^2/(4p)} e^{i q P}
 *                * sum_{k1<=i, k2<=j} C(i,k1) C(j,k2) s_A^{i-k1} s_B^{j-k2} m_{k1+k2},
 *         s_A = P - A + i q/(2p),  s_B = P - B + i q/(2p),
 *         m_{2n} = (2n-1)!!/(2p)^n,  m_odd = 0.
 *     This is the same integral the paper reduces with its b-coefficients
 *     and Hermite polynomials (Sec. 4, eqs. sigmaTidbits, positionTidbits,
 *     bCoefficients, Mij, CartesianVector); it is computed here by a
 *     different route so that the two can check each other.
 *  5. Omega_{mu nu}(q) = c_mu c_nu sum_{k,l} d_k d_l n_k n_l I_x I_y I_z.
 *  6. f_s(q) = s_f sum_{mu,nu} T^s_{mu nu} Omega_{mu nu}(q); OpenMP over q.
 *
 * FFT method (Sec. 3, eq. PhiTDM; Sec. 5.2): the transition density on
 * points, written out from its definition in the AO basis,
 *     Phi_s(r) = s_f sum_{mu,nu} T^s_{mu nu} phi_mu(r) phi_nu(r),
 *     phi_mu(r) = c_mu sum_k d_k n_k (x-A_x)^a (y-A_y)^b (z-A_z)^c e^{-alpha_k |r-A|^2}
 * (App. A primitives with the normalisations of steps 2-3), FP64, no
 * thresholding; OpenMP over points.  The transform itself is done in the
 * Python wrapper with a library FFT.
 *
 * Pins (tests that tie this file to something other than itself) are listed
 * in the test suite: same-centre s/p/d closed forms, 1D and 3D real-space
 * quadrature, the paper's Hermite form, and the invariants f(-q) = f(q)*,
 * translation, signed-permutation rotation, f(0) = s_f Tr(T S), linearity,
 * f(T) = f(T^T), inversion parity and the low-q dipole limit.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int atom;
    int pw[3];      /* Cartesian powers (a, b, c) */
    int prim_off;   /* first primitive in exps/coefs */
    int nprim;
    double c;       /* contracted normalisation */
} comp_t;

static const int CART[3][6][3] = {
    {{0, 0, 0}},
    {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}},
    {{2, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}},
};

static int ncart(int l) { return (l + 1) * (l + 2) / 2; }

/* n!! with (-1)!! = 0!! = 1 */
static double dfact(int n) {
    double r = 1.0;
    for (int k = n; k > 1; k -= 2) r *= (double)k;
    return r;
}

static double binom(int n, int k) {
    double r = 1.0;
    for (int t = 1; t <= k; ++t) r = r * (double)(n - k + t) / (double)t;
    return r;
}

static double complex cipow(double complex z, int n) {
    double complex r = 1.0;
    for (int k = 0; k < n; ++k) r *= z;
    return r;
}

/* step 2: unit self-overlap of x^a y^b z^c exp(-alpha r^2) */
static double prim_norm(double alpha, const int pw[3]) {
    double s = 1.0;
    for (int ax = 0; ax < 3; ++ax)
        s *= dfact(2 * pw[ax] - 1) / pow(4.0 * alpha, pw[ax]) * sqrt(M_PI / (2.0 * alpha));
    return 1.0 / sqrt(s);
}

/* step 3: self-overlap of the contracted component before rescaling */
static double contracted_self_overlap(const comp_t* m, const double* exps, const double* coefs) {
    double s = 0.0;
    for (int k = 0; k < m->nprim; ++k)
        for (int l = 0; l < m->nprim; ++l) {
            double a = exps[m->prim_off + k], b = exps[m->prim_off + l];
            double p = a + b, t = 1.0;
            for (int ax = 0; ax < 3; ++ax)
                t *= dfact(2 * m->pw[ax] - 1) / pow(2.0 * p, m->pw[ax]) * sqrt(M_PI / p);
            s += coefs[m->prim_off + k] * coefs[m->prim_off + l] * prim_norm(a, m->pw) *
                 prim_norm(b, m->pw) * t;
        }
    return s;
}

/* step 4: the 1D integral for one primitive pair and one axis */
static double complex axis_integral(int i, int j, double A, double B, double alpha,
                                    double beta, double q) {
    double p = alpha + beta;
    double P = (alpha * A + beta * B) / p;
    double complex sA = (P - A) + I * (q / (2.0 * p));
    double complex sB = (P - B) + I * (q / (2.0 * p));
    double complex sum = 0.0;
    for (int k1 = 0; k1 <= i; ++k1)
        for (int k2 = 0; k2 <= j; ++k2) {
            int t = k1 + k2;
            if (t & 1) continue;
            double mom = dfact(t - 1) / pow(2.0 * p, t / 2);
            sum += binom(i, k1) * binom(j, k2) * cipow(sA, i - k1) * cipow(sB, j - k2) * mom;
        }
    double pre = sqrt(M_PI / p) * exp(-alpha * beta / p * (A - B) * (A - B)) *
                 exp(-q * q / (4.0 * p));
    return pre * cexp(I * (q * P)) * sum;
}

static int build_components(int n_shells, const int* shell_atom, const int* shell_l,
                            const int* shell_nprim, const double* exps, const double* coefs,
                            int normalise, comp_t** out) {
    int nbf = 0;
    for (int s = 0; s < n_shells; ++s) {
        if (shell_l[s] < 0 || shell_l[s] > 2 || shell_nprim[s] <= 0) return -1;
        nbf += ncart(shell_l[s]);
    }
    comp_t* comp = (comp_t*)calloc((size_t)nbf, sizeof(comp_t));
    if (!comp) return -2;
    int mu = 0, off = 0;
    for (int s = 0; s < n_shells; ++s) {
        for (int c = 0; c < ncart(shell_l[s]); ++c, ++mu) {
            comp[mu].atom = shell_atom[s];
            memcpy(comp[mu].pw, CART[shell_l[s]][c], sizeof(int) * 3);
            comp[mu].prim_off = off;
            comp[mu].nprim = shell_nprim[s];
            comp[mu].c = 1.0;
        }
        off += shell_nprim[s];
    }
    if (normalise)
        for (int m = 0; m < nbf; ++m)
            comp[m].c = 1.0 / sqrt(contracted_self_overlap(&comp[m], exps, coefs));
    *out = comp;
    return nbf;
}

/* step 5 */
static double complex omega(const comp_t* m, const comp_t* n, const double* xyz,
                            const double* exps, const double* coefs, const double* q) {
    const double* A = xyz + 3 * m->atom;
    const double* B = xyz + 3 * n->atom;
    double complex acc = 0.0;
    for (int k = 0; k < m->nprim; ++k)
        for (int l = 0; l < n->nprim; ++l) {
            double a = exps[m->prim_off + k], b = exps[n->prim_off + l];
            double w = coefs[m->prim_off + k] * coefs[n->prim_off + l] * prim_norm(a, m->pw) *
                       prim_norm(b, n->pw);
            double complex v = w;
            for (int ax = 0; ax < 3; ++ax)
                v *= axis_integral(m->pw[ax], n->pw[ax], A[ax], B[ax], a, b, q[ax]);
            acc += v;
        }
    return m->c * n->c * acc;
}

/* Number of Cartesian basis functions; negative on bad shells. */
int scffo_nbf(int n_shells, const int* shell_l) {
    int nbf = 0;
    for (int s = 0; s < n_shells; ++s) {
        if (shell_l[s] < 0 || shell_l[s] > 2) return -1;
        nbf += ncart(shell_l[s]);
    }
    return nbf;
}

/* Contracted normalisation constants c_mu (step 3), [nbf]. */
int scffo_norms(int n_shells, const int* shell_atom, const int* shell_l, const int* shell_nprim,
                const double* exps, const double* coefs, double* c_out) {
    comp_t* comp = NULL;
    int nbf = build_components(n_shells, shell_atom, shell_l, shell_nprim, exps, coefs, 1, &comp);
    if (nbf < 0) return nbf;
    for (int m = 0; m < nbf; ++m) c_out[m] = comp[m].c;
    free(comp);
    return 0;
}

/*
 * Step 6.  f_out is [n_states][n_q][2] (re, im) doubles; q is [n_q][3] (a.u.);
 * T is [n_states][nbf][nbf] row-major.  n_threads <= 0 uses the OpenMP default.
 * Returns 0, or a negative code for malformed shells.
 */
int scffo_eval(int n_atoms, const double* xyz, int n_shells, const int* shell_atom,
               const int* shell_l, const int* shell_nprim, const double* exps,
               const double* coefs, int normalise, int n_states, const double* T, int n_q,
               const double* q, double spin_factor, double* f_out, int n_threads) {
    (void)n_atoms;
    comp_t* comp = NULL;
    int nbf = build_components(n_shells, shell_atom, shell_l, shell_nprim, exps, coefs,
                               normalise, &comp);
    if (nbf < 0) return nbf;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int iq = 0; iq < n_q; ++iq) {
        double complex* fs = (double complex*)calloc((size_t)(n_states > 0 ? n_states : 1),
                                                     sizeof(double complex));
        for (int m = 0; m < nbf; ++m)
            for (int n = 0; n < nbf; ++n) {
                double complex om = omega(&comp[m], &comp[n], xyz, exps, coefs, q + 3 * iq);
                for (int s = 0; s < n_states; ++s)
                    fs[s] += T[((size_t)s * nbf + m) * nbf + n] * om;
            }
        for (int s = 0; s < n_states; ++s) {
            f_out[((size_t)s * n_q + iq) * 2 + 0] = spin_factor * creal(fs[s]);
            f_out[((size_t)s * n_q + iq) * 2 + 1] = spin_factor * cimag(fs[s]);
        }
        free(fs);
    }
    free(comp);
    return 0;
}

/* Omega_{mu nu}(q) for every component pair at one q: out is [nbf][nbf][2]. */
int scffo_pair_matrix(int n_atoms, const double* xyz, int n_shells, const int* shell_atom,
                      const int* shell_l, const int* shell_nprim, const double* exps,
                      const double* coefs, int normalise, const double* q, double* out) {
    (void)n_atoms;
    comp_t* comp = NULL;
    int nbf = build_components(n_shells, shell_atom, shell_l, shell_nprim, exps, coefs,
                               normalise, &comp);
    if (nbf < 0) return nbf;
    for (int m = 0; m < nbf; ++m)
        for (int n = 0; n < nbf; ++n) {
            double complex om = omega(&comp[m], &comp[n], xyz, exps, coefs, q);
            out[((size_t)m * nbf + n) * 2 + 0] = creal(om);
            out[((size_t)m * nbf + n) * 2 + 1] = cimag(om);
        }
    free(comp);
    return 0;
}

/* phi_mu(r) of every component at one point (App. A primitive sum) */
static void ao_values(const comp_t* comp, int nbf, const double* xyz, const double* exps,
                      const double* coefs, const double* r, double* phi) {
    for (int m = 0; m < nbf; ++m) {
        const double* A = xyz + 3 * comp[m].atom;
        double d[3], r2 = 0.0, mono = 1.0;
        for (int ax = 0; ax < 3; ++ax) {
            d[ax] = r[ax] - A[ax];
            r2 += d[ax] * d[ax];
            for (int e = 0; e < comp[m].pw[ax]; ++e) mono *= d[ax];
        }
        double rad = 0.0;
        for (int k = 0; k < comp[m].nprim; ++k) {
            double a = exps[comp[m].prim_off + k];
            rad += coefs[comp[m].prim_off + k] * prim_norm(a, comp[m].pw) * exp(-a * r2);
        }
        phi[m] = comp[m].c * mono * rad;
    }
}

/*
 * Transition density (FFT method, eq. PhiTDM in the AO basis).  r is
 * [n_pts][3] (bohr); phi_out is [n_states][n_pts];  T as in scffo_eval.
 */
int scffo_density(int n_atoms, const double* xyz, int n_shells, const int* shell_atom,
                  const int* shell_l, const int* shell_nprim, const double* exps,
                  const double* coefs, int normalise, int n_states, const double* T, int n_pts,
                  const double* r, double spin_factor, double* phi_out, int n_threads) {
    (void)n_atoms;
    comp_t* comp = NULL;
    int nbf = build_components(n_shells, shell_atom, shell_l, shell_nprim, exps, coefs,
                               normalise, &comp);
    if (nbf < 0) return nbf;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel
    {
        double* phi = (double*)malloc(sizeof(double) * (size_t)nbf);
#pragma omp for schedule(static)
        for (int ip = 0; ip < n_pts; ++ip) {
            ao_values(comp, nbf, xyz, exps, coefs, r + 3 * (size_t)ip, phi);
            for (int s = 0; s < n_states; ++s) {
                const double* Ts = T + (size_t)s * nbf * nbf;
                double acc = 0.0;
                for (int m = 0; m < nbf; ++m)
                    for (int n = 0; n < nbf; ++n) acc += Ts[(size_t)m * nbf + n] * phi[m] * phi[n];
                phi_out[(size_t)s * n_pts + ip] = spin_factor * acc;
            }
        }
        free(phi);
    }
    free(comp);
    return 0;
}

/* phi_mu at each point: out is [n_pts][nbf]. */
int scffo_ao_values(int n_atoms, const double* xyz, int n_shells, const int* shell_atom,
                    const int* shell_l, const int* shell_nprim, const double* exps,
                    const double* coefs, int normalise, int n_pts, const double* r, double* out) {
    (void)n_atoms;
    comp_t* comp = NULL;
    int nbf = build_components(n_shells, shell_atom, shell_l, shell_nprim, exps, coefs,
                               normalise, &comp);
    if (nbf < 0) return nbf;
    for (int ip = 0; ip < n_pts; ++ip)
        ao_values(comp, nbf, xyz, exps, coefs, r + 3 * (size_t)ip, out + (size_t)ip * nbf);
    free(comp);
    return 0;
}
