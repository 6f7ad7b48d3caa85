// Drives the library's host code on the mock runtime: the serving engine
// (several submitting threads, mixed request kinds and precisions, polls,
// takes, releases), a batch call from another thread at the same time, then
// context teardown with requests never taken.  Exit status 0 when every
// status is as expected and the mock reported nothing.
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "../../include/shssa.h"

extern "C" int mock_audit_errors();

static std::atomic<int> g_bad{0};
static std::atomic<int> g_nomem{0};
// with a device memory cap (MOCK_DEVICE_BYTES) running out of memory is an
// expected outcome, reported as SSA_ENOMEM
static const bool g_capped = std::getenv("MOCK_DEVICE_BYTES") != nullptr;

static void expect(bool ok, const char* what, int code) {
    if (!ok && g_capped && code == SSA_ENOMEM) {
        g_nomem++;
        return;
    }
    if (!ok) {
        g_bad++;
        std::fprintf(stderr, "DRIVER: %s (status %d: %s)\n", what, code, ssa_last_error());
    }
}

static void client(ssa_ctx* ctx, int id, int nreq, bool take_all) {
    std::mt19937 rng(1234u + (unsigned)id);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    std::vector<uint64_t> tickets;
    std::vector<int> ngs;
    std::vector<size_t> nout;
    const int gp[4] = {0, 2, 4, 5}, gi[5] = {0, 1, 2, 3, 0};
    for (int k = 0; k < nreq; ++k) {
        const double u = U(rng);
        const int prec = U(rng) < 0.6 ? SSA_FP32 : SSA_FP64;
        const int r = 4 + (int)(U(rng) * 6);   // groups use components 0..3
        uint64_t t = 0;
        int rc;
        size_t cells;
        if (u < 0.5) {   // series
            const int n = 300 + (int)(U(rng) * 1500);
            std::vector<double> x(n);
            for (int i = 0; i < n; ++i) x[i] = std::sin(i * 0.1) + 0.1 * U(rng);
            ssa_request q{x.data(), n, 1, nullptr, nullptr, n / 2, 1, r, prec, 7ull + k};
            rc = ssa_submit(ctx, &q, gp, gi, 3, &t);
            cells = (size_t)n;
        } else if (u < 0.75) {   // MSSA
            const int s = 2 + (int)(U(rng) * 4);
            std::vector<std::vector<double>> ser(s);
            std::vector<const double*> ptr(s);
            std::vector<int> len(s);
            int nmax = 0;
            for (int j = 0; j < s; ++j) {
                len[j] = 200 + (int)(U(rng) * 300);
                nmax = std::max(nmax, len[j]);
                ser[j].resize(len[j]);
                for (int i = 0; i < len[j]; ++i) ser[j][i] = std::cos(i * 0.05 * (j + 1)) + 0.1 * U(rng);
                ptr[j] = ser[j].data();
            }
            rc = ssa_submit_multi(ctx, ptr.data(), len.data(), s, 100, r, prec, gp, gi, 3, &t);
            cells = (size_t)s * nmax;
        } else {   // image
            const int side = 48 + (int)(U(rng) * 80);
            std::vector<double> x((size_t)side * side);
            for (size_t i = 0; i < x.size(); ++i) x[i] = std::sin(0.03 * (double)i) + 0.1 * U(rng);
            ssa_request q{x.data(), side, side, nullptr, nullptr, side / 6, side / 6, r, prec, 11ull + k};
            rc = ssa_submit(ctx, &q, gp, gi, 3, &t);
            cells = (size_t)side * side;
        }
        expect(rc == SSA_OK, "submit", rc);
        if (rc != SSA_OK) continue;
        tickets.push_back(t);
        ngs.push_back(3);
        nout.push_back(cells);
        if (U(rng) < 0.3) std::this_thread::sleep_for(std::chrono::microseconds((int)(U(rng) * 3000)));
    }
    // take all (or, for one client, leave the last few for the context teardown)
    const size_t ntake = take_all ? tickets.size() : tickets.size() / 2;
    for (size_t k = 0; k < ntake; ++k) {
        int done = 0;
        ssa_poll(ctx, tickets[k], &done);
        int rc = ssa_wait(ctx, tickets[k]);
        expect(rc == SSA_OK, "wait", rc);
        ssa_decomp* d = nullptr;
        std::vector<double> rec(nout[k] * (size_t)ngs[k] * 2);
        ssa_times tm{};
        rc = ssa_take(ctx, tickets[k], &d, rec.data(), &tm);
        expect(rc == SSA_OK, "take", rc);
        if (d) {
            if (k % 3 == 0) {   // use the handle after its batch's stream moved on
                const int g2p[2] = {0, 1}, g2i[1] = {0};
                std::vector<double> out(nout[k] * 2);
                const int rr = ssa_reconstruct(d, g2p, g2i, 1, out.data());
                expect(rr == SSA_OK, "reconstruct after take", rr);
            }
            ssa_free(d);
        }
    }
}

static void batcher(ssa_ctx* ctx, int rounds) {
    for (int k = 0; k < rounds; ++k) {
        const int n = 5;
        std::vector<std::vector<double>> xs(n);
        std::vector<ssa_request> q(n);
        for (int i = 0; i < n; ++i) {
            const int side = 40 + 8 * i;
            xs[i].resize((size_t)side * side);
            for (size_t c = 0; c < xs[i].size(); ++c) xs[i][c] = std::cos(0.02 * (double)c * (i + 1));
            q[i] = ssa_request{xs[i].data(), side, side, nullptr, nullptr, 8, 8, 4, k % 2 ? SSA_FP64 : SSA_FP32,
                               99ull + (unsigned)i};
        }
        std::vector<ssa_decomp*> out(n, nullptr);
        std::vector<int> st(n, -1);
        const int rc = ssa_decompose_batch(ctx, n, q.data(), out.data(), st.data());
        expect(rc == SSA_OK, "batch call", rc);
        for (int i = 0; i < n; ++i) {
            expect(st[i] == SSA_OK, "batch member", st[i]);
            if (out[i]) ssa_free(out[i]);
        }
    }
}

// The other entry points on handles made in this thread (the mock's data
// are not numbers the methods would meet: only the host side is checked
// here, so their statuses are reported, not required, except that none may
// report a runtime failure).
static void extras(ssa_ctx* ctx) {
    const bool verbose = std::getenv("AUDIT_VERBOSE") != nullptr;
    auto ok = [verbose](int rc, const char* what) {
        if (verbose) std::fprintf(stderr, "extras: %s -> %d\n", what, rc);
        expect(rc != SSA_EDEVICE, what, rc);
    };
    // 1D series
    const int n = 600;
    std::vector<double> x(n);
    for (int i = 0; i < n; ++i) x[i] = std::sin(0.2 * i) + 0.01 * i;
    ssa_decomp* d = nullptr;
    int rc = ssa_decompose(ctx, x.data(), n, 1, nullptr, nullptr, 200, 1, 6, SSA_FP64, &d);
    ok(rc, "decompose series");
    if (d) {
        const int gp[3] = {0, 2, 4}, gi[4] = {0, 1, 2, 3}, grp[2] = {0, 1};
        std::vector<double> rho(4), contrib(2), out(4 * n), re(2), im(2), fc(100);
        int ns = 0;
        ok(ssa_wcor(d, gp, gi, 2, rho.data(), contrib.data()), "wcor");
        ok(ssa_rforecast(d, grp, 2, 50, fc.data(), &ns), "rforecast");
        ok(ssa_vforecast(d, grp, 2, 50, fc.data(), &ns), "vforecast");
        ok(ssa_esprit(d, grp, 2, re.data(), im.data()), "esprit");
        ok(ssa_esprit_tls(d, grp, 2, re.data(), im.data()), "esprit tls");
        ok(ssa_esprit_noalloc(d, grp, 2, re.data(), im.data()), "esprit noalloc");
        ok(ssa_reconstruct(d, gp, gi, 2, out.data()), "reconstruct");
        ok(ssa_extend(d, 9), "extend");
        ok(ssa_reconstruct(d, gp, gi, 2, out.data()), "reconstruct after extend");
        ssa_free(d);
    }
    // image: eigen method (small and blocked windows), vectors, weights, 2D-ESPRIT, row forecasts
    const int side = 64;
    std::vector<double> img((size_t)side * side);
    for (size_t i = 0; i < img.size(); ++i) img[i] = std::cos(0.07 * (double)(i % side)) * std::sin(0.05 * (double)(i / side));
    for (int lw : {8, 14}) {
        ssa_decomp* e = nullptr;
        rc = ssa_decompose_eigen(ctx, img.data(), side, side, nullptr, nullptr, lw, lw, 4, &e);
        ok(rc, "decompose eigen");
        if (e) {
            const int grp[2] = {0, 1};
            std::vector<double> U(4 * lw * lw), V(4 * (size_t)(side - lw + 1) * (side - lw + 1)), w(img.size());
            std::vector<double> a(2), b(2), c(2), dd(2), fc(4 * 100);
            int ns = 0;
            ok(ssa_get_vectors(e, U.data(), V.data()), "vectors");
            ok(ssa_get_weights(e, w.data()), "weights");
            ok(ssa_esprit2d(e, grp, 2, a.data(), b.data(), c.data(), dd.data()), "esprit2d");
            ok(ssa_rforecast_row(e, grp, 2, 5, nullptr, &ns), "row forecast size");
            ok(ssa_extend(e, 6), "extend eigen");
            ssa_free(e);
        }
    }
    // a series longer than one transform row (decomposed in segments)
    {
        const int nl = 41000;
        std::vector<double> xl(nl);
        for (int i = 0; i < nl; ++i) xl[i] = std::sin(0.17 * i) + 0.001 * (i % 97);
        ssa_decomp* ls = nullptr;
        ok(ssa_decompose(ctx, xl.data(), nl, 1, nullptr, nullptr, 40, 1, 4, SSA_FP64, &ls), "decompose long series");
        if (ls) {
            const int gp[3] = {0, 2, 4}, gi[4] = {0, 1, 2, 3};
            std::vector<double> rec(2 * (size_t)nl), w(nl), rho(4), U(4 * 40), V(4 * (size_t)(nl - 39));
            ok(ssa_reconstruct(ls, gp, gi, 2, rec.data()), "reconstruct long series");
            ok(ssa_get_weights(ls, w.data()), "weights long series");
            ok(ssa_get_vectors(ls, U.data(), V.data()), "vectors long series");
            ok(ssa_wcor(ls, gp, gi, 2, rho.data(), nullptr), "wcor long series");
            ssa_free(ls);
        }
    }
    // MSSA and M-2D packings
    std::vector<std::vector<double>> ser(3, std::vector<double>(300));
    std::vector<const double*> sp(3);
    std::vector<int> len(3, 300);
    for (int j = 0; j < 3; ++j) {
        for (int i = 0; i < 300; ++i) ser[j][i] = std::sin(0.1 * i * (j + 1));
        sp[j] = ser[j].data();
    }
    ssa_decomp* m = nullptr;
    ok(ssa_decompose_multi(ctx, sp.data(), len.data(), 3, 100, 4, SSA_FP32, &m), "decompose multi");
    if (m) ssa_free(m);
    std::vector<const double*> ims{img.data(), img.data()};
    std::vector<int> nxs{side, side}, nys{side, side}, off(2);
    ssa_decomp* m2 = nullptr;
    ok(ssa_decompose_m2d(ctx, ims.data(), nxs.data(), nys.data(), 2, nullptr, 8, 8, 4, SSA_FP32, off.data(), &m2),
       "decompose m2d");
    if (m2) ssa_free(m2);
}

int main(int argc, char** argv) {
    // the serving threads (SHSSA_SERVE_ENGINE), or with AUDIT_COOP the
    // cooperative server that the clients' waits drive
    if (!std::getenv("AUDIT_COOP")) setenv("SHSSA_SERVE_ENGINE", "1", 1);
    const int nreq = argc > 1 ? std::atoi(argv[1]) : 40;
    const size_t budget = argc > 2 ? (size_t)std::strtoull(argv[2], nullptr, 10) : 0;
    // the length tuner and the tune cache file run too (AUDIT_TUNE_CACHE: its path)
    const char* cache = std::getenv("AUDIT_TUNE_CACHE");
    if (cache) setenv("SHSSA_LEN_TUNE", "1", 1);
    ssa_ctx* ctx = nullptr;
    int rc = ssa_ctx_create(0, budget, cache, &ctx);
    if (rc != SSA_OK) {
        std::fprintf(stderr, "DRIVER: context creation failed: %s\n", ssa_last_error());
        return 2;
    }
    std::thread c1(client, ctx, 1, nreq, true);
    std::thread c2(client, ctx, 2, nreq, false);
    std::thread bt(batcher, ctx, 3);
    std::thread ex(extras, ctx);
    c1.join();
    c2.join();
    bt.join();
    ex.join();
    ssa_ctx_destroy(ctx);   // requests of client 2 never taken are released here
    const int audit = mock_audit_errors();
    std::printf("driver: %d unexpected statuses, %d out of memory, %d audit reports\n", g_bad.load(),
                g_nomem.load(), audit);
    return (g_bad.load() || audit) ? 1 : 0;
}
