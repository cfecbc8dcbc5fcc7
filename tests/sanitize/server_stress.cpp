// Host-side stress of the request server in its scheduler test mode
// (device = -1: no GPU; requests are validated, admitted under the budget,
// batched and completed, nothing is computed).  Built with ThreadSanitizer
// or AddressSanitizer + UndefinedBehaviorSanitizer on the host code by
// run.sh.  Several submitter threads, random cancellations, malformed
// requests (rejected at submit or failing in prep), statistics readers,
// and destruction with requests still queued.  Exit status 0 when every
// ticket ends in a consistent state.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "scarff.h"

namespace {

struct Mol {
    std::vector<double> xyz, exps, coefs, T;
    std::vector<int> sa, sl, sn;
    int nbf = 0;
};

Mol make_mol(std::mt19937_64& g, bool bad) {
    std::uniform_real_distribution<double> u(0.0, 1.0);
    Mol m;
    const int na = 1 + (int)(g() % 4);
    for (int a = 0; a < na; ++a)
        for (int k = 0; k < 3; ++k) m.xyz.push_back(4.0 * u(g));
    const int ns = 1 + (int)(g() % 6);
    for (int s = 0; s < ns; ++s) {
        const int l = (int)(g() % 3), np = 1 + (int)(g() % 3);
        m.sa.push_back((int)(g() % na));
        m.sl.push_back(l);
        m.sn.push_back(np);
        for (int p = 0; p < np; ++p) {
            m.exps.push_back(0.1 + 50.0 * u(g));
            m.coefs.push_back(0.1 + u(g));
        }
        m.nbf += (l + 1) * (l + 2) / 2;
    }
    if (bad) m.exps[0] = -1.0;   // fails in prep (basis validation)
    return m;
}

}  // namespace

int main() {
    scff_server* srv = nullptr;
    const size_t budget = 3u << 20;
    if (scff_server_create(-1, budget, 4, &srv) != SCFF_OK) {
        std::fprintf(stderr, "create: %s\n", scff_last_error());
        return 1;
    }
    std::atomic<int> bad_state{0}, done_ok{0}, done_fail{0}, cancelled{0}, rejected{0};
    std::atomic<bool> stop_stats{false};
    std::thread stats([&] {
        scff_server_stats st;
        while (!stop_stats.load())
            if (scff_server_stats_get(srv, &st) != SCFF_OK || st.admitted_bytes > st.budget_bytes) bad_state++;
    });
    auto submitter = [&](int id) {
        std::mt19937_64 g(1000 + id);
        std::vector<unsigned long long> tickets;
        std::vector<std::vector<float>> outs;
        for (int i = 0; i < 60; ++i) {
            const bool bad = (i % 13) == 7;
            Mol m = make_mol(g, bad);
            const int nst = 1 + (int)(g() % 4);
            m.T.assign((size_t)nst * m.nbf * m.nbf, 0.01);
            const int N = 4 + (int)(g() % 8);
            outs.emplace_back((size_t)nst * N * N * N * 3);
            scff_request r{};
            r.n_atoms = (int)m.xyz.size() / 3;
            r.xyz_bohr = m.xyz.data();
            r.n_shells = (int)m.sa.size();
            r.shell_atom = m.sa.data();
            r.shell_l = m.sl.data();
            r.shell_nprim = m.sn.data();
            r.exps = m.exps.data();
            r.coefs = m.coefs.data();
            r.normalise = 1;
            r.n_states = (i % 17) == 5 ? 0 : nst;   // rejected at submit
            r.T = m.T.data();
            for (int a = 0; a < 3; ++a) {
                r.grid.n[a] = N;
                r.grid.qmin[a] = -4.0;
                r.grid.qmax[a] = 4.0;
            }
            r.precision = SCFF_FP32;
            r.f = outs.back().data();
            r.f2 = outs.back().data() + (size_t)nst * N * N * N * 2;
            unsigned long long t = 0;
            if (scff_server_submit(srv, &r, &t) != SCFF_OK) {
                rejected++;
                continue;
            }
            tickets.push_back(t);
            if (g() % 5 == 0) (void)scff_server_cancel(srv, t);   // may be too late: SCFF_EBUSY
        }
        for (unsigned long long t : tickets) {
            int st = 0;
            long long lat = 0;
            if (scff_server_wait(srv, t, -1, &st, &lat) != SCFF_OK) {
                bad_state++;
                continue;
            }
            if (st == SCFF_OK) done_ok++;
            else if (st == SCFF_ECANCELLED) cancelled++;
            else if (st == SCFF_EINVAL) done_fail++;
            else bad_state++;
        }
    };
    std::vector<std::thread> th;
    for (int i = 0; i < 4; ++i) th.emplace_back(submitter, i);
    for (auto& t : th) t.join();
    stop_stats = true;
    stats.join();
    // a second server destroyed with requests still queued
    scff_server* srv2 = nullptr;
    if (scff_server_create(-1, budget, 2, &srv2) == SCFF_OK) {
        std::mt19937_64 g(7);
        std::vector<std::vector<float>> outs;
        std::vector<Mol> keep;
        for (int i = 0; i < 20; ++i) {
            keep.push_back(make_mol(g, false));
            Mol& m = keep.back();
            m.T.assign((size_t)m.nbf * m.nbf, 0.01);
            outs.emplace_back(8 * 8 * 8 * 3);
            scff_request r{};
            r.n_atoms = (int)m.xyz.size() / 3;
            r.xyz_bohr = m.xyz.data();
            r.n_shells = (int)m.sa.size();
            r.shell_atom = m.sa.data();
            r.shell_l = m.sl.data();
            r.shell_nprim = m.sn.data();
            r.exps = m.exps.data();
            r.coefs = m.coefs.data();
            r.normalise = 1;
            r.n_states = 1;
            r.T = m.T.data();
            for (int a = 0; a < 3; ++a) {
                r.grid.n[a] = 8;
                r.grid.qmin[a] = -3.0;
                r.grid.qmax[a] = 3.0;
            }
            r.f = outs.back().data();
            unsigned long long t = 0;
            (void)scff_server_submit(srv2, &r, &t);
        }
        scff_server_destroy(srv2);
    }
    scff_server_stats st;
    scff_server_stats_get(srv, &st);
    scff_server_destroy(srv);
    std::printf("ok %d, failed %d, cancelled %d, rejected %d, inconsistent %d; batches %lld for %lld requests\n",
                done_ok.load(), done_fail.load(), cancelled.load(), rejected.load(), bad_state.load(), st.batches,
                st.batched_requests);
    return bad_state.load() == 0 && done_ok.load() > 0 ? 0 : 1;
}
