// Internal declarations of the form-factor engine (host precompute, device
// kernels, runtime).  Not part of the public ABI; see include/scarff.h.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/scarff.h"

namespace scff {

// Maximum primitive-pair terms per (virtual) component pair.  A component
// pair with more terms is split into several virtual pairs that share its
// packed transition weight, so any contraction length is supported.
constexpr int kMaxTermsPerPair = 9;
// Component pairs processed per staging step of the grid kernel.
constexpr int kChunk = 8;
// States per MFMA row block.
constexpr int kStateBlock = 16;
constexpr int kMaxStates = 32;
constexpr int kMaxPrim = 32;

// One 1D V-tensor row: a (primitive pair, axis, power pair) triple.  On a
// q value of its axis it evaluates
//   V(q) = exp(-q^2/(4p)) * exp(i q P) * sum_u e[u] (i q)^u ,
// where every q-independent factor of the pair (contraction coefficients,
// primitive normalisation on this axis, sqrt(pi/p) and the Gaussian product
// prefactor; on the x row also the remaining axes' prefactors) is folded
// into e[].
struct VRow {
    double p;        // alpha + beta
    double P;        // product centre on this axis
    double e[5];     // polynomial coefficients, u = 0..deg
    int axis;
    int deg;         // i + j
};

// Device copy of a row.  The 1D tables are built from it in FP64 and rounded
// once to FP32 (phase argument, range reduction, Gaussian and polynomial).
struct VRowDev {
    double P;
    double inv4p;    // 1/(4p)
    double e[5];
    int deg;
    int axis;
};

struct Term {        // one (component pair, primitive pair) term
    int row[3];
    double bound;    // q-independent bound of |V^x V^y V^z| over all q
};

struct CompPair {
    int mu, nu;
    int first_term, n_terms;
};

struct Basis {
    int n_atoms = 0, n_shells = 0, nbf = 0;
    std::vector<double> xyz;
    std::vector<int> sh_atom, sh_l, sh_nprim, sh_off, sh_bf0;
    std::vector<double> exps, coefs;
    std::vector<double> cnorm;   // contracted normalisation per AO
    std::vector<int> bf_shell;   // shell of each AO
    std::vector<int> bf_pw;      // 3 powers per AO
    bool normalise = true;
};

struct PairData {               // q- and T-independent pair precompute
    std::vector<VRow> rows;
    std::vector<Term> terms;
    std::vector<CompPair> cps;
    long long shell_pairs = 0;
    long long prim_pairs_total = 0;   // sum over component pairs of primitive pairs
};

// Result of screening + packing for one (molecule, T, options) state.
struct Packed {
    int n_states = 0;
    int state_blocks = 1;              // 16-row MFMA blocks (1 or 2)
    int n_vpairs = 0;                  // virtual component pairs (padded to kChunk)
    int n_chunks = 0;
    std::vector<int> chunk_off;        // offset of chunk c in `terms`
    std::vector<int> chunk_npp;        // terms per virtual pair in chunk c
    std::vector<int> terms;            // [chunk][kChunk][npp] x 4 ints (rowx,rowy,rowz,valid)
    std::vector<VRowDev> rows;         // compacted rows referenced by kept terms
    std::vector<float> tp;             // [n_vpairs][16*state_blocks]
    std::vector<uint16_t> tp_hi, tp_lo;   // split-BF16 copies of tp
    long long pairs_kept = 0;          // K
    long long terms_kept = 0;          // R
    long long pairs_total = 0;
};

// ---- host precompute (precompute.cpp) ----
std::string build_basis(Basis& b, int n_atoms, const double* xyz, int n_shells,
                        const int* shell_atom, const int* shell_l, const int* shell_nprim,
                        const double* exps, const double* coefs, int normalise);
void build_pairs(const Basis& b, PairData& pd);
std::string pack(const Basis& b, const PairData& pd, int n_states, const double* T,
                 double screen_eps, double spin_factor, Packed& out);
uint16_t bf16_rne(float x);
float bf16_to_float(uint16_t h);

// ---- runtime.cpp ----
// Thread-local message returned by scff_last_error().
void set_error(const std::string& msg);
// Pack and upload a context's problem for grid g; *bytes_needed receives the
// device bytes an evaluation on g will hold in total.
int ctx_prepare(scff_ctx* c, const scff_grid* g, size_t* bytes_needed);

}  // namespace scff
