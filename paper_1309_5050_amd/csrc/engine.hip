// Host engine and C ABI of the Shaped 2D-SSA library.
//
// A request is validated and mapped to an internal grid (see common.hpp),
// then requests of equal geometry, rank and precision run as one batch:
// every kernel launch covers all instances of the batch, which advance in
// lockstep through the bidiagonalisation cycles (instances that converge
// drop out at the next cycle boundary).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/shssa.h"
#include "common.hpp"
#include "device.hpp"
#include "launch.hpp"

#ifdef SHSSA_HOST_AUDIT
// Host audit build (tests only, with the mock runtime): called whenever a
// device block becomes free for reuse; the mock reports queued work that
// still uses it (reuse_on: the stream that reuses it at once, whose own
// queue is ordered behind the earlier uses).
extern "C" void shssa_audit_block(const void* p, size_t n, hipStream_t reuse_on);
extern "C" void shssa_audit_take(const void* p, size_t n);   // a pooled block leaves the pool
#endif

using namespace shssa;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(call)                                                                                  \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess) return fail(SSA_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point t) {
    return std::chrono::duration<double, std::milli>(Clock::now() - t).count();
}

// Row kernel selector: size class (bits 0..2), power-of-two plan (bit 3)
// and, for powers of two, log2 of the half-length (bits 4..7).
int row_word(int nh, bool f64) {
    int w = row_class(nh, f64);
    if (nh > 0 && (nh & (nh - 1)) == 0) {
        int lg = 0;
        while ((1 << lg) < nh) ++lg;
        w |= 8 | (lg << 4);
    }
    return w;
}

int next_smooth(int n) {
    for (int m = std::max(n, 1);; ++m) {
        int t = m;
        for (int p : {2, 3, 5, 7})
            while (t % p == 0) t /= p;
        if (t == 1) return m;
    }
}

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

bool make_plan(int n, FftPlan& pl) {
    pl.n = n;
    pl.npass = 0;
    int t = n;
    auto take = [&](int r) {
        while (t % r == 0 && pl.npass < kMaxPass) {
            pl.radix[pl.npass++] = (int8_t)r;
            t /= r;
        }
    };
    take(8); take(4); take(2); take(3); take(5); take(7);
    return t == 1;
}

bool make_plan_ok(int n) {
    FftPlan pl;
    return make_plan(n, pl);
}

}  // namespace

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------

struct Server;   // serving state (asynchronous requests), created on first submit

// Transform lengths chosen by the length tuner, process-wide (every context
// then pads a size class alike, so results agree across contexts):
// (kind 0 = row half-length / 1 = column length, f64, natural length) ->
// chosen length.
std::mutex g_len_mu;
std::map<std::tuple<int, int, int>, int> g_len_tc;

// Chosen length for a natural length n0, and whether the class is tuned.
std::pair<int, bool> len_choice(int kind, bool f64, int n0) {
    std::lock_guard<std::mutex> g(g_len_mu);
    auto it = g_len_tc.find(std::make_tuple(kind, (int)f64, n0));
    return it == g_len_tc.end() ? std::make_pair(n0, false) : std::make_pair(it->second, true);
}

// The power-of-two alternative to a natural transform length (0 if none):
// rows (half-lengths) up to 512, the register kernels' range, columns up
// to 1024; at most 30% more points.
int len_alternative(int kind, int n0, int need) {
    int p = 1;
    while (p < need) p <<= 1;
    if (p == n0 || p > (kind == 0 ? 512 : 1024) || 10 * p > 13 * n0) return 0;
    return p;
}

struct ssa_ctx {
    int device = 0;
    std::atomic<Server*> srv{nullptr};   // started by the first ssa_submit (under srv_mu)
    std::mutex srv_mu;
    // Entry points that queue work on the context's stream run one at a
    // time: they share the stream and its staging and readback buffers.
    std::recursive_mutex call_mu;
    int refs = 0;            // live decompositions (guarded by mu)
    bool closing = false;    // ssa_ctx_destroy called; delete when refs drops to 0
    hipStream_t st = nullptr;
    bool own = false;
    std::vector<hipStream_t> sub_st;   // streams of concurrent sub-batches (created on demand)
    size_t budget = 0;
    size_t used = 0;
    std::mutex mu;
    std::map<std::tuple<int, int, int>, void*> tw;   // (n, f64, real split) -> table
    std::map<std::pair<int, int>, int> col_tc;       // (f64, MA) -> tuned column tile
    std::mutex tune_mu;                               // one tuning at a time; guards col_tc
    std::string tune_path;                            // autotune cache file ("" = none)
    int slots = 0;                                    // continuous batching: instances advancing together (0 = all)
    bool len_tune = false;                            // length tuner on (SHSSA_LEN_TUNE at creation)

    // Tuning results persist in a text file, one choice per line:
    //   col <f64> <MA> <config>         column tile and kernel variant
    //   rowlen <f64> <nh0> <nh>         row half-length for a natural one
    //   collen <f64> <MA0> <MA>         column length for a natural one
    // Lines of another kind or with a configuration this build does not
    // compile are ignored when used.  Caller holds tune_mu.
    void tune_load() {
        if (tune_path.empty()) return;
        FILE* f = std::fopen(tune_path.c_str(), "r");
        if (!f) return;
        char kind[16];
        int a = 0, b = 0, c = 0;
        char line[256];
        while (std::fgets(line, sizeof line, f)) {
            if (std::sscanf(line, "%15s %d %d %d", kind, &a, &b, &c) != 4) continue;
            if (std::strcmp(kind, "col") == 0) col_tc[std::make_pair(a, b)] = c;
            if (std::strcmp(kind, "rowlen") == 0 || std::strcmp(kind, "collen") == 0) {
                std::lock_guard<std::mutex> g(g_len_mu);
                g_len_tc[std::make_tuple(kind[0] == 'r' ? 0 : 1, a, b)] = c;
            }
        }
        std::fclose(f);
    }
    void tune_save(const char* kind, int a, int b, int c) {
        if (tune_path.empty()) return;
        if (FILE* f = std::fopen(tune_path.c_str(), "a")) {
            std::fprintf(f, "%s %d %d %d\n", kind, a, b, c);
            std::fclose(f);
        }
    }

    int tile_for(bool f64, int MA) {
        std::lock_guard<std::mutex> g(tune_mu);
        auto it = col_tc.find(std::make_pair((int)f64, MA));
        return it != col_tc.end() ? it->second : col_tile(f64);
    }
    // kernel timing (see ssa_ctx_profile)
    std::vector<std::string> prof_kinds;   // kernel classes being timed
    std::vector<long> prof_seen;           // launches of each class since timing started
    int prof_every = 1;                    // time one launch in every prof_every of a class
    std::vector<hipEvent_t> ev_pool;
    struct Span {
        int e0, e1, kind;
        double bytes;
    };
    std::vector<Span> spans;
    int prof_index(const char* kind) const {
        for (size_t k = 0; k < prof_kinds.size(); ++k)
            if (prof_kinds[k] == kind) return (int)k;
        return -1;
    }

    // A step about to run launches counts[i].second kernels of class
    // counts[i].first.  True if one of them is in the timing sample (the
    // step then runs with its spans, which count the launches); otherwise
    // the launches are counted here as run untimed.
    bool prof_take_step(const std::vector<std::pair<const char*, int>>& counts, int steps = 1) {
        std::lock_guard<std::mutex> g(mu);
        if (prof_kinds.empty()) return false;
        for (auto& c : counts) {
            const int k = prof_index(c.first);
            if (k < 0) continue;
            for (int i = 0; i < c.second * steps; ++i)
                if ((prof_seen[k] + i) % prof_every == 0) return true;
        }
        for (auto& c : counts) {
            const int k = prof_index(c.first);
            if (k >= 0) prof_seen[k] += c.second * steps;
        }
        return false;
    }

    // next unused event of the pool (caller holds mu); reset by profile_read
    int ev_next = 0;
    hipEvent_t prof_ref = nullptr;   // recorded when timing starts: the common time origin
    int prof_event() {
        const int k = ev_next;
        while ((int)ev_pool.size() <= k) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return -1;
            ev_pool.push_back(e);
        }
        ++ev_next;
        return k;
    }

    // Device memory pool: freed blocks are kept per size class and handed
    // out again, so steady-state work never calls hipMalloc/hipFree (hipFree
    // synchronises the device).
    std::map<size_t, std::vector<void*>> pool;
    size_t pooled = 0;

    static size_t size_class(size_t b) {
        if (b <= 4096) return 4096;
        const int lg = 63 - __builtin_clzll(b);
        const size_t q = (size_t)1 << (lg - 2);
        return (b + q - 1) / q * q;
    }
    // caller holds mu
    bool nopool = std::getenv("SHSSA_NO_POOL") != nullptr;
    void* pool_get(size_t cls) {
        if (nopool) {
            void* p = nullptr;
            return hipMalloc(&p, cls) == hipSuccess ? p : nullptr;
        }
        auto it = pool.find(cls);
        if ((it == pool.end() || it->second.empty()) && !deferred.empty()) {
            reclaim();
            it = pool.find(cls);
        }
        if (it != pool.end() && !it->second.empty()) {
            void* p = it->second.back();
            it->second.pop_back();
            pooled -= cls;
#ifdef SHSSA_HOST_AUDIT
            shssa_audit_take(p, cls);
#endif
            return p;
        }
        void* p = nullptr;
        if (hipMalloc(&p, cls) != hipSuccess) {
            // release the pool and try once more
            for (auto& kv : pool)
                for (void* q : kv.second) {
#ifdef SHSSA_HOST_AUDIT
                    shssa_audit_take(q, kv.first);
#endif
                    (void)hipFree(q);
                }
            pool.clear();
            pooled = 0;
            if (hipMalloc(&p, cls) != hipSuccess) return nullptr;
        }
        return p;
    }
    void pool_put(void* p, size_t cls) {
#ifdef SHSSA_HOST_AUDIT
        shssa_audit_block(p, cls, nullptr);
#endif
        if (nopool) {
            (void)hipFree(p);
            return;
        }
        pool[cls].push_back(p);
        pooled += cls;
    }

    // Blocks whose last users may still be queued on a stream go back to
    // the pool once an event recorded after those users has completed, so
    // library calls return without waiting for their work (caller holds mu).
    struct Deferred {
        hipEvent_t ev;
        std::vector<std::pair<void*, size_t>> blocks;
    };
    std::vector<Deferred> deferred;
    std::vector<hipEvent_t> spare_ev;
    void defer(std::vector<std::pair<void*, size_t>>& blocks, hipStream_t s) {
        if (blocks.empty()) return;
        hipEvent_t e = nullptr;
        if (!spare_ev.empty()) {
            e = spare_ev.back();
            spare_ev.pop_back();
        } else if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            e = nullptr;
        }
        if (!e || hipEventRecord(e, s) != hipSuccess) {
            // no event: wait for the stream instead
            (void)hipStreamSynchronize(s);
            for (auto& b : blocks) pool_put(b.first, b.second);
            if (e) spare_ev.push_back(e);
        } else {
            deferred.push_back(Deferred{e, {}});
            deferred.back().blocks.swap(blocks);
        }
        blocks.clear();
    }
    // as defer, behind an event the caller recorded (ownership moves here)
    void defer_ev(std::vector<std::pair<void*, size_t>>& blocks, hipEvent_t e) {
        deferred.push_back(Deferred{e, {}});
        deferred.back().blocks.swap(blocks);
        blocks.clear();
    }
    hipEvent_t take_event() {
        if (!spare_ev.empty()) {
            hipEvent_t e = spare_ev.back();
            spare_ev.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        return hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess ? e : nullptr;
    }
    void reclaim() {
        size_t k = 0;
        for (size_t i = 0; i < deferred.size(); ++i) {
            if (hipEventQuery(deferred[i].ev) == hipSuccess) {
                for (auto& b : deferred[i].blocks) pool_put(b.first, b.second);
                spare_ev.push_back(deferred[i].ev);
            } else {
                if (k != i) deferred[k] = std::move(deferred[i]);
                ++k;
            }
        }
        deferred.resize(k);
    }

    // Pinned host staging for uploads, one per stream.  Two halves are
    // filled in turn; a half is refilled only after the copies issued from it
    // have completed (an event recorded when it was left), so hipMemcpyAsync
    // from it never blocks the host and never reads overwritten data.
    static constexpr size_t kStageHalf = 8u << 20;
    struct Stage {
        char* buf = nullptr;
        size_t head = 0;
        int cur = 0;
        hipEvent_t ev[2] = {nullptr, nullptr};
        bool pending[2] = {false, false};
    };
    std::map<hipStream_t, Stage> stages;   // guarded by mu

    int upload_locked(void* dst, const void* src, size_t n, hipStream_t s) {
        if (n == 0) return SSA_OK;
        const size_t need = (n + 255) & ~(size_t)255;
        if (need > kStageHalf) {
            // too large to stage: a plain (host-synchronous) copy
            HIPCHK(hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, s));
            HIPCHK(hipStreamSynchronize(s));
            return SSA_OK;
        }
        Stage& g = stages[s];
        if (!g.buf) {
            HIPCHK(hipHostMalloc((void**)&g.buf, 2 * kStageHalf, hipHostMallocDefault));
            HIPCHK(hipEventCreateWithFlags(&g.ev[0], hipEventDisableTiming));
            HIPCHK(hipEventCreateWithFlags(&g.ev[1], hipEventDisableTiming));
        }
        if (g.head + need > kStageHalf) {
            HIPCHK(hipEventRecord(g.ev[g.cur], s));
            g.pending[g.cur] = true;
            g.cur ^= 1;
            g.head = 0;
            if (g.pending[g.cur]) {
                HIPCHK(hipEventSynchronize(g.ev[g.cur]));
                g.pending[g.cur] = false;
            }
        }
        char* h = g.buf + (size_t)g.cur * kStageHalf + g.head;
        std::memcpy(h, src, n);
        g.head += need;
        HIPCHK(hipMemcpyAsync(dst, h, n, hipMemcpyHostToDevice, s));
        return SSA_OK;
    }
    int upload(void* dst, const void* src, size_t n, hipStream_t s) {
        std::lock_guard<std::mutex> g(mu);
        return upload_locked(dst, src, n, s);
    }
    // A stream is about to be destroyed: wait for its copies, drop its stage.
    void stage_drop(hipStream_t s) {
        std::lock_guard<std::mutex> g(mu);
        auto it = stages.find(s);
        if (it == stages.end()) return;
        (void)hipStreamSynchronize(s);
        if (it->second.buf) (void)hipHostFree(it->second.buf);
        for (auto e : it->second.ev)
            if (e) (void)hipEventDestroy(e);
        stages.erase(it);
    }
    void stage_free() {
        for (auto& kv : stages) {
            if (kv.second.buf) (void)hipHostFree(kv.second.buf);
            for (auto e : kv.second.ev)
                if (e) (void)hipEventDestroy(e);
        }
        stages.clear();
    }

    // Pinned host buffers for batched readbacks, one per stream (grown on
    // demand; a stream's readbacks are synchronous, so one buffer suffices).
    std::map<hipStream_t, std::pair<void*, size_t>> rbs;   // guarded by mu
    int readback_buf(hipStream_t s, size_t n, void** out) {
        std::lock_guard<std::mutex> g(mu);
        auto& rb = rbs[s];
        if (n > rb.second) {
            if (rb.first) (void)hipHostFree(rb.first);
            rb.first = nullptr;
            rb.second = 0;
            HIPCHK(hipHostMalloc(&rb.first, n, hipHostMallocDefault));
            rb.second = n;
        }
        *out = rb.first;
        return SSA_OK;
    }
    void readback_free() {
        for (auto& kv : rbs)
            if (kv.second.first) (void)hipHostFree(kv.second.first);
        rbs.clear();
    }

    // twiddles exp(-2 pi i t / N) for t = 0..cnt-1 (N = n, or 2n for the split)
    int twiddles(int n, bool f64, bool split, const void** out) {
        std::lock_guard<std::mutex> lock(mu);
        auto key = std::make_tuple(n, (int)f64, (int)split);
        auto it = tw.find(key);
        if (it != tw.end()) {
            *out = it->second;
            return SSA_OK;
        }
        const int cnt = split ? n + 1 : n;
        const long double N = split ? 2.0L * n : (long double)n;
        std::vector<double> d(2 * (size_t)cnt);
        for (int t = 0; t < cnt; ++t) {
            const long double a = -2.0L * 3.14159265358979323846264338327950288L * t / N;
            d[2 * t] = (double)cosl(a);
            d[2 * t + 1] = (double)sinl(a);
        }
        void* p = nullptr;
        const size_t bytes = (size_t)cnt * (f64 ? 16 : 8);
        if (hipMalloc(&p, bytes) != hipSuccess) return fail(SSA_ENOMEM, "device memory (twiddle table)");
        if (f64) {
            HIPCHK(hipMemcpy(p, d.data(), bytes, hipMemcpyHostToDevice));
        } else {
            std::vector<float> f(d.begin(), d.end());
            HIPCHK(hipMemcpy(p, f.data(), bytes, hipMemcpyHostToDevice));
        }
        tw[key] = p;
        *out = p;
        return SSA_OK;
    }
};

// ---------------------------------------------------------------------------
// one decomposition
// ---------------------------------------------------------------------------

struct ssa_decomp {
    ssa_ctx* ctx = nullptr;
    // A series too long for one transform row (Alg. 1 allows any length):
    // the handle holds the MSSA decomposition of overlapping segments,
    // segment p = x[p B .. p B + B + L - 2], whose L x B trajectory matrices
    // side by side are the series' own L x K matrix (columns p B .. p B + B
    // - 1 each), so sigma and U are the series'.  The getters return the
    // series' layout: V concatenated over the segments, weights and
    // reconstructions summed over every segment that holds a value
    // (diagonal averaging over the whole matrix).
    struct Seg {
        bool on = false;
        bool col = true;              // series given as N x 1 (else 1 x N)
        int N = 0, L = 0, B = 0, s = 0, nmax = 0;
        std::vector<double> x;        // the series, NaN where missing
    } seg;
    // caller geometry
    int nx = 0, ny = 0, lx = 0, ly = 0, kx = 0, ky = 0;
    bool tr = false;                 // internal grid is the transpose
    // internal geometry
    int A = 0, B = 0, LA = 0, LB = 0, KA = 0, KB = 0, MA = 1, MB = 0, nh = 0, P = 0, ldp = 0;
    int nh0 = 0, MA0 = 1;            // natural (smooth) transform lengths before the tuner's choice
    bool rowfam = false, f64 = true;
    bool eigen = false;              // eigen method: S = X X^T and its eigenpairs
    double* Sbig = nullptr;          // eigen method beyond kMaxBasis cells: S, then its rotated columns (L x L)
    double* eig_lam = nullptr;       // |columns| of the rotated S: the eigenvalues (L)
    std::vector<double> eig_lam_h;   // host copy of eig_lam
    int r = 0;
    unsigned long long seed = 0;
    long L = 0, K = 0;
    int side = 0;
    long nshort = 0, nlong = 0;
    int status = SSA_OK;
    bool decomposed = false;
    std::vector<uint8_t> lmask_h;    // internal LA x LB
    std::vector<int> lrow_h;         // LA + 1
    std::vector<int> ra, rb0, rb1;   // window runs (internal)
    std::vector<uint8_t> kmask_h;    // internal KA x KB (fetched on demand)
    std::vector<double> sigma_h;     // filled from the device on first request
    bool sigma_ready = false;
    // Work queued on this handle: inside a library call the stream it went
    // to (last_st); when a call returns, an event recorded behind it
    // (last_ev), which stays valid whatever happens to the stream later.
    hipStream_t last_st = nullptr;
    hipEvent_t last_ev = nullptr;
    // device memory (blocks of the context pool, with their size class)
    std::vector<std::pair<void*, size_t>> allocs;
    size_t bytes = 0;
    double *x = nullptr, *xc = nullptr, *W = nullptr;
    uint8_t *mask = nullptr, *nset = nullptr, *kmask = nullptr, *lmask = nullptr;
    int *npref = nullptr, *kpref = nullptr, *lpref = nullptr, *kcount = nullptr, *krow = nullptr, *lrow = nullptr, *runs = nullptr;
    void *Xh = nullptr, *T1 = nullptr, *T2 = nullptr, *Us = nullptr;
    long tslot = 0, uslot = 0;
    double *Q = nullptr, *w = nullptr, *sinv = nullptr, *hp1 = nullptr, *hp2 = nullptr, *np = nullptr, *np0 = nullptr;
    double *lnp = nullptr, *gam = nullptr, *Bm = nullptr, *Yl = nullptr, *Yr = nullptr, *sig = nullptr, *beta = nullptr;
    double* Qtmp = nullptr;
    float* Q32 = nullptr;            // FP32 copy of Q for the reorthogonalisation (SSA_FP32_BASIS32)
    bool q32 = false;                // the reorthogonalisation reads the FP32 copy
    void* lbuf = nullptr;
    int *perm = nullptr, *flag = nullptr;
    double *U = nullptr, *V = nullptr, *sigma = nullptr;
    OpDesc op{};
    LzDesc lz{};
    ResDesc rs{};
    Runs rn{};
    ssa_stats st{};

    ~ssa_decomp();
    void attach(ssa_ctx* c) {
        ctx = c;
        std::lock_guard<std::mutex> g(c->mu);
        c->refs++;
    }

    template <typename T>
    int dalloc(T** p, size_t count) {
        const size_t cls = ssa_ctx::size_class(std::max<size_t>(count, 1) * sizeof(T));
        std::lock_guard<std::mutex> g(ctx->mu);
        if (ctx->budget && ctx->used + cls > ctx->budget)
            return fail(SSA_ENOMEM, "device memory budget exhausted");
        void* q = ctx->pool_get(cls);
        if (!q) return fail(SSA_ENOMEM, "hipMalloc failed");
        ctx->used += cls;
        allocs.push_back({q, cls});
        bytes += cls;
        *p = static_cast<T*>(q);
        return SSA_OK;
    }

    // Returns block p of the handle to the pool once the work queued on s
    // has completed.
    void dfree(void* p, hipStream_t s) {
        if (!p) return;
        std::lock_guard<std::mutex> g(ctx->mu);
        for (size_t i = 0; i < allocs.size(); ++i) {
            if (allocs[i].first != p) continue;
            std::vector<std::pair<void*, size_t>> one{allocs[i]};
            bytes -= allocs[i].second;
            ctx->used -= std::min(ctx->used, allocs[i].second);
            allocs.erase(allocs.begin() + (long)i);
            ctx->defer(one, s);
            return;
        }
    }

    size_t celem() const { return f64 ? 16 : 8; }
};

namespace {

// Context of the calling thread's current library call: the pool that small
// batch tables come from (set by every entry point that makes them).
thread_local ssa_ctx* g_tables_ctx = nullptr;

void ctx_release(ssa_ctx* ctx) {
    if (g_tables_ctx == ctx) g_tables_ctx = nullptr;
    (void)hipStreamSynchronize(ctx->st);
    for (auto x : ctx->sub_st) (void)hipStreamSynchronize(x);
    for (auto& df : ctx->deferred) {
        (void)hipEventSynchronize(df.ev);
        for (auto& b : df.blocks) (void)hipFree(b.first);
        (void)hipEventDestroy(df.ev);
    }
    for (auto e : ctx->spare_ev) (void)hipEventDestroy(e);
    for (auto& kv : ctx->tw) (void)hipFree(kv.second);
    for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
    if (ctx->prof_ref) (void)hipEventDestroy(ctx->prof_ref);
    for (auto& kv : ctx->pool)
        for (void* q : kv.second) (void)hipFree(q);
    for (auto x : ctx->sub_st) (void)hipStreamSynchronize(x);
    ctx->stage_free();
    ctx->readback_free();
    for (auto x : ctx->sub_st) (void)hipStreamDestroy(x);
    if (ctx->own) (void)hipStreamDestroy(ctx->st);
    delete ctx;
}

}  // namespace

// A handle returns its device blocks to the context pool; the context itself
// is released with its last handle once ssa_ctx_destroy has been called.
ssa_decomp::~ssa_decomp() {
    if (!ctx) return;
    bool last = false;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        if (last_ev) {
            ctx->defer_ev(allocs, last_ev);   // queued work may still use the blocks
            last_ev = nullptr;
        } else if (last_st) {
            ctx->defer(allocs, last_st);
        } else {
            for (auto& a : allocs) ctx->pool_put(a.first, a.second);
        }
        ctx->used -= std::min(ctx->used, bytes);
        ctx->refs--;
        last = ctx->closing && ctx->refs == 0;
    }
    if (last) ctx_release(ctx);
}

namespace {

// Validate a request and compute the internal geometry (host side only).
int plan_request(ssa_ctx* ctx, const ssa_request& q, ssa_decomp* d, int nh_force = 0, int ma_force = 0) {
    if (q.nx <= 0 || q.ny <= 0 || q.lx <= 0 || q.ly <= 0) return fail(SSA_EINVAL, "sizes must be positive");
    if (!q.x) return fail(SSA_EINVAL, "x is NULL");
    if (q.precision != SSA_FP64 && q.precision != SSA_FP32 && q.precision != SSA_FP32_BASIS32)
        return fail(SSA_EINVAL, "unknown precision");
    d->attach(ctx);
    d->nx = q.nx;
    d->ny = q.ny;
    d->r = q.r;
    d->seed = q.seed;
    d->f64 = q.precision == SSA_FP64;
    d->q32 = q.precision == SSA_FP32_BASIS32;
    // window: trim to the bounding box
    int i0 = q.lx, i1 = -1, j0 = q.ly, j1 = -1;
    for (int i = 0; i < q.lx; ++i)
        for (int j = 0; j < q.ly; ++j)
            if (!q.wmask || q.wmask[(long)i * q.ly + j]) {
                i0 = std::min(i0, i); i1 = std::max(i1, i);
                j0 = std::min(j0, j); j1 = std::max(j1, j);
            }
    if (i1 < 0) return fail(SSA_EINVAL, "empty window");
    d->lx = i1 - i0 + 1;
    d->ly = j1 - j0 + 1;
    if (d->lx > q.nx || d->ly > q.ny) return fail(SSA_EINVAL, "window box exceeds the array");
    if ((long)d->lx * d->ly <= 1 || (long)d->lx * d->ly >= (long)q.nx * q.ny)
        return fail(SSA_EINVAL, "window box must satisfy 1 < Lx*Ly < Nx*Ny");
    d->kx = q.nx - d->lx + 1;
    d->ky = q.ny - d->ly + 1;
    // orientation: a window one column wide is turned into one row high so
    // that the cross-row part of the product is a plain sum.
    d->tr = d->ly == 1 && d->lx > 1;
    d->A = d->tr ? q.ny : q.nx;
    d->B = d->tr ? q.nx : q.ny;
    d->LA = d->tr ? d->ly : d->lx;
    d->LB = d->tr ? d->lx : d->ly;
    d->KA = d->A - d->LA + 1;
    d->KB = d->B - d->LB + 1;
    d->rowfam = d->LA == 1;
    // window mask in the internal orientation, row offsets and runs
    d->lmask_h.assign((size_t)d->LA * d->LB, 0);
    for (int i = 0; i < d->lx; ++i)
        for (int j = 0; j < d->ly; ++j) {
            const bool in = !q.wmask || q.wmask[(long)(i + i0) * q.ly + (j + j0)];
            const int a = d->tr ? j : i, b = d->tr ? i : j;
            d->lmask_h[(size_t)a * d->LB + b] = in;
        }
    d->lrow_h.assign(d->LA + 1, 0);
    d->ra.clear(); d->rb0.clear(); d->rb1.clear();
    for (int a = 0; a < d->LA; ++a) {
        int cnt = 0;
        for (int b = 0; b < d->LB;) {
            if (!d->lmask_h[(size_t)a * d->LB + b]) { ++b; continue; }
            int e = b;
            while (e < d->LB && d->lmask_h[(size_t)a * d->LB + e]) ++e;
            d->ra.push_back(a); d->rb0.push_back(b); d->rb1.push_back(e);
            cnt += e - b;
            b = e;
        }
        d->lrow_h[a + 1] = d->lrow_h[a] + cnt;
    }
    d->L = d->lrow_h[d->LA];
    // transform sizes
    // transform sizes: any M >= N gives the same products and averages, so
    // the natural (2,3,5,7-smooth) length or the tuner's choice for it
    d->nh0 = next_smooth((d->B + 1) / 2);
    d->nh = nh_force > 0 ? nh_force : ctx->len_tune ? len_choice(0, d->f64, d->nh0).first : d->nh0;
    if (d->nh < (d->B + 1) / 2 || !make_plan_ok(d->nh)) d->nh = d->nh0;
    d->MB = 2 * d->nh;
    d->P = d->nh + 1;
    d->ldp = (d->P + 15) / 16 * 16;   // 128-byte aligned column tiles
    if (row_class(d->nh, d->f64) < 0) return fail(SSA_EINVAL, "row length beyond the supported transform size");
    if (!d->rowfam) {
        d->MA0 = next_smooth(d->A);
        d->MA = ma_force > 0 ? ma_force : ctx->len_tune ? len_choice(1, d->f64, d->MA0).first : d->MA0;
        if (d->MA < d->A || !make_plan_ok(d->MA)) d->MA = d->MA0;
        if (d->MA > 1024) return fail(SSA_EINVAL, "column length beyond the supported transform size (1024)");
    } else {
        d->MA = 1;
    }
    if (q.r < 1) return fail(SSA_ERANK, "r must be >= 1");
    if (q.r > kMaxRank) return fail(SSA_ERANK, "r must be <= 120 (the basis holds 128 vectors)");
    return SSA_OK;
}

// Upload the request's data in the internal orientation.  With jobs, the
// device-to-device copies of device inputs are queued there for one batched
// launch (which the caller issues before any kernel reads the copies).
int upload_request(const ssa_request& q, ssa_decomp* d, bool dev_input, hipStream_t st,
                   std::vector<CopyJob>* jobs = nullptr) {
    const long n = (long)d->A * d->B;
    int rc;
    d->last_st = st;
    if ((rc = d->dalloc(&d->x, n))) return rc;
    if (q.mask && (rc = d->dalloc(&d->mask, n))) return rc;
    if (dev_input) {
        if (!d->tr || d->nx == 1 || d->ny == 1) {
            if (jobs) jobs->push_back({q.x, d->x, n * 8});
            else HIPCHK(hipMemcpyAsync(d->x, q.x, n * 8, hipMemcpyDeviceToDevice, st));
        } else {
            launch_transpose(1, d->nx, d->ny, st, q.x, d->x);
        }
        if (q.mask) {
            if (d->tr && d->nx > 1 && d->ny > 1) {
                std::vector<uint8_t> hm(n), tm(n);
                HIPCHK(hipMemcpyAsync(hm.data(), q.mask, n, hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
                for (int i = 0; i < d->nx; ++i)
                    for (int j = 0; j < d->ny; ++j) tm[(size_t)j * d->nx + i] = hm[(size_t)i * d->ny + j];
                if ((rc = d->ctx->upload(d->mask, tm.data(), n, st))) return rc;
            } else if (jobs) {
                jobs->push_back({q.mask, d->mask, n});
            } else {
                HIPCHK(hipMemcpyAsync(d->mask, q.mask, n, hipMemcpyDeviceToDevice, st));
            }
        }
    } else {
        if (!d->tr) {
            if ((rc = d->ctx->upload(d->x, q.x, n * 8, st))) return rc;
            if (q.mask && (rc = d->ctx->upload(d->mask, q.mask, n, st))) return rc;
        } else {
            std::vector<double> tx(n);
            for (int i = 0; i < d->nx; ++i)
                for (int j = 0; j < d->ny; ++j) tx[(size_t)j * d->nx + i] = q.x[(size_t)i * d->ny + j];
            if ((rc = d->ctx->upload(d->x, tx.data(), n * 8, st))) return rc;
            std::vector<uint8_t> tm;
            if (q.mask) {
                tm.resize(n);
                for (int i = 0; i < d->nx; ++i)
                    for (int j = 0; j < d->ny; ++j) tm[(size_t)j * d->nx + i] = q.mask[(size_t)i * d->ny + j];
                if ((rc = d->ctx->upload(d->mask, tm.data(), n, st))) return rc;
            }
        }
    }
    // shape buffers
    if ((rc = d->dalloc(&d->nset, n))) return rc;
    if ((rc = d->dalloc(&d->xc, n))) return rc;
    if ((rc = d->dalloc(&d->npref, (long)d->A * (d->B + 1)))) return rc;
    if ((rc = d->dalloc(&d->kmask, (long)d->KA * d->KB))) return rc;
    if ((rc = d->dalloc(&d->kpref, (long)d->KA * (d->KB + 1)))) return rc;
    if ((rc = d->dalloc(&d->kcount, d->KA))) return rc;
    if ((rc = d->dalloc(&d->krow, d->KA + 1))) return rc;
    if ((rc = d->dalloc(&d->W, n))) return rc;
    const bool lfull = d->L == (long)d->LA * d->LB;
    // The window's tables in one block and one upload: row offsets, runs
    // and, for a shaped window, the per-row exclusive prefix counts and the
    // mask bytes (from a 256-byte boundary).
    const int nrun = (int)d->ra.size();
    const size_t o_runs = (size_t)d->LA + 1;
    const size_t o_pref = o_runs + 3 * (size_t)nrun;
    const size_t n_pref = lfull ? 0 : (size_t)d->LA * (d->LB + 1);
    const size_t o_mask = (o_pref + n_pref + 63) / 64 * 64;
    const size_t n_mask = lfull ? 0 : ((size_t)d->LA * d->LB + 3) / 4;
    std::vector<int> tab(o_mask + n_mask, 0);
    std::copy(d->lrow_h.begin(), d->lrow_h.end(), tab.begin());
    std::copy(d->ra.begin(), d->ra.end(), tab.begin() + o_runs);
    std::copy(d->rb0.begin(), d->rb0.end(), tab.begin() + o_runs + nrun);
    std::copy(d->rb1.begin(), d->rb1.end(), tab.begin() + o_runs + 2 * (size_t)nrun);
    if (!lfull) {
        for (int a = 0; a < d->LA; ++a) {
            int* pr = tab.data() + o_pref + (size_t)a * (d->LB + 1);
            for (int b = 0; b < d->LB; ++b) pr[b + 1] = pr[b] + d->lmask_h[(size_t)a * d->LB + b];
        }
        std::memcpy(tab.data() + o_mask, d->lmask_h.data(), d->lmask_h.size());
    }
    int* blk = nullptr;
    if ((rc = d->dalloc(&blk, tab.size()))) return rc;
    if ((rc = d->ctx->upload(blk, tab.data(), tab.size() * sizeof(int), st))) return rc;
    d->lrow = blk;
    d->runs = blk + o_runs;
    if (!lfull) {
        d->lpref = blk + o_pref;
        d->lmask = reinterpret_cast<uint8_t*>(blk + o_mask);
    }
    d->rn = Runs{d->runs, d->runs + nrun, d->runs + 2 * nrun, nrun, d->L};
    // descriptor (K set filled after the origin count)
    OpDesc& o = d->op;
    o.A = d->A; o.B = d->B; o.MA = d->MA; o.MB = d->MB; o.P = d->P; o.ldp = d->ldp;
    o.rowfam = d->rowfam;
    o.spec_scale = d->rowfam ? 1.0 / d->MB : 1.0 / ((double)d->MA * d->MB);
    o.S[0] = CellSet{d->LA, d->LB, d->L, lfull ? nullptr : d->lmask, d->lrow, lfull ? nullptr : d->lpref};
    o.S[1] = CellSet{d->KA, d->KB, 0, d->kmask, d->krow, d->kpref};
    o.W = d->W;
    o.xc = d->xc;
    o.nset = d->nset;
    return SSA_OK;
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------

// (g_tables_ctx, the pool that small batch tables come from, is declared
// with the context release)
// Table blocks released by a serving worker stay with that worker (its
// stream may still read them) until the worker has synchronised its stream;
// then flush_table_cache returns them to the context pool.
thread_local std::vector<std::pair<void*, size_t>>* g_table_cache = nullptr;

void flush_table_cache(ssa_ctx* ctx) {
    if (!g_table_cache) return;
    std::lock_guard<std::mutex> g(ctx->mu);
    for (auto& b : *g_table_cache) ctx->pool_put(b.first, b.second);
    g_table_cache->clear();
}

// Scope of a library call on stream st: table blocks released inside it
// return to the shared pool only after the work queued on st so far has
// completed (serving workers on other streams share the pool); the call
// itself does not wait.
struct TableScope {
    ssa_ctx* ctx;
    hipStream_t st;
    std::vector<std::pair<void*, size_t>> cache;
    bool owner = false;
    TableScope(ssa_ctx* c, hipStream_t s) : ctx(c), st(s) {
        if (!g_table_cache) {
            g_table_cache = &cache;
            owner = true;
        }
    }
    ~TableScope() {
        if (!owner) return;
        {
            std::lock_guard<std::mutex> g(ctx->mu);
            ctx->defer(cache, st);
        }
        g_table_cache = nullptr;
    }
};

// A small device table filled from the host (descriptor arrays, item lists).
struct DevVec {
    void* p = nullptr;
    size_t cap = 0;
    ssa_ctx* ctx = nullptr;   // context of the calling thread's library call, bound at first use
    DevVec() = default;
    int bind() {
        if (!ctx) ctx = g_tables_ctx;
        return ctx ? SSA_OK : fail(SSA_EINVAL, "device tables outside a library call");
    }
    // a block has one owner: a copy would return it to the pool twice
    DevVec(const DevVec&) = delete;
    DevVec& operator=(const DevVec&) = delete;
    ~DevVec() { release(); }
    void release() {
        if (!p) return;
        if (g_table_cache) {
            g_table_cache->push_back({p, cap});
        } else {
            std::lock_guard<std::mutex> g(ctx->mu);
            ctx->pool_put(p, cap);
        }
        p = nullptr;
        cap = 0;
    }
    template <typename T>
    int put(const std::vector<T>& v, hipStream_t st) {
        if (int rc = bind()) return rc;
        const size_t b = ssa_ctx::size_class(std::max<size_t>(v.size(), 1) * sizeof(T));
        if (b > cap) {
            release();
            if (g_table_cache) {
                for (size_t k = 0; k < g_table_cache->size(); ++k)
                    if ((*g_table_cache)[k].second == b) {
                        p = (*g_table_cache)[k].first;
                        g_table_cache->erase(g_table_cache->begin() + k);
#ifdef SHSSA_HOST_AUDIT
                        shssa_audit_block(p, b, st);   // reused on st: only other streams must be done
#endif
                        break;
                    }
            }
            if (!p) {
                std::lock_guard<std::mutex> g(ctx->mu);
                p = ctx->pool_get(b);
            }
            if (!p) return fail(SSA_ENOMEM, "hipMalloc (batch tables)");
            cap = b;
        }
        return ctx->upload(p, v.data(), v.size() * sizeof(T), st);
    }
    template <typename T> T* as() const { return static_cast<T*>(p); }
    // device space without contents (from the pool)
    int reserve(size_t bytes) {
        if (int rc = bind()) return rc;
        const size_t b = ssa_ctx::size_class(std::max<size_t>(bytes, 1));
        if (b <= cap) return SSA_OK;
        release();
        {
            std::lock_guard<std::mutex> g(ctx->mu);
            p = ctx->pool_get(b);
        }
        if (!p) return fail(SSA_ENOMEM, "device memory (work buffer)");
        cap = b;
        return SSA_OK;
    }
};

struct ItemList {
    std::vector<Item> h;
    DevVec d;
    const Item* dp = nullptr;   // device copy inside another list's table (upload_lists)
    int n() const { return (int)h.size(); }
    const Item* ptr() const { return dp ? dp : d.as<Item>(); }
    int upload(hipStream_t st) {
        dp = nullptr;
        return d.put(h, st);
    }
};

// Several item lists in one host-to-device copy: the first list's table
// holds them all, the others point into it (valid while the first lives and
// is not uploaded again).
int upload_lists(std::initializer_list<ItemList*> ls, hipStream_t st) {
    ItemList* own = *ls.begin();
    std::vector<Item> all;
    std::vector<size_t> off;
    for (ItemList* L : ls) {
        off.push_back(all.size());
        all.insert(all.end(), L->h.begin(), L->h.end());
    }
    const int rc = own->d.put(all, st);
    if (rc) return rc;
    size_t k = 0;
    for (ItemList* L : ls) L->dp = own->d.as<Item>() + off[k++];
    return SSA_OK;
}

// Host tables of mixed types packed into one device block (one copy).
struct TablePack {
    std::vector<char> h;
    DevVec d;
    template <typename T>
    size_t add(const std::vector<T>& v) {
        const size_t off = (h.size() + 15) & ~size_t(15);
        h.resize(off + std::max<size_t>(v.size(), 1) * sizeof(T));
        if (!v.empty()) std::memcpy(h.data() + off, v.data(), v.size() * sizeof(T));
        return off;
    }
    int upload(hipStream_t st) { return d.put(h, st); }
    template <typename T> T* at(size_t off) const { return reinterpret_cast<T*>(static_cast<char*>(d.p) + off); }
};

struct Batch {
    ssa_ctx* ctx;
    hipStream_t st;
    std::vector<ssa_decomp*> ds;      // instance i = ds[i]
    bool f64 = true, rowfam = false;
    int cls = 0, TC = 16, CV = 0;   // row size class (| 8: radix-2/4/8 plan), column tile and variant
    DevVec dops, dlz, dres, druns;
    std::vector<OpDesc> hops;
    std::vector<LzDesc> hlz;
    std::vector<ResDesc> hres;
    std::vector<Runs> hruns;
    // per-batch scratch for the convergence flags; the step counter
    // [j, jstart] read by replayed steps
    DevVec dflag, dstep;

    explicit Batch(ssa_ctx* c) : ctx(c), st(c->st) {}
    // The handles outlive the batch: its step counter (released with it) must
    // not stay in their descriptors.  Queued work keeps the uploaded copies.
    ~Batch() {
        const int* c = dstep.as<int>();
        for (auto* d : ds)
            if (d && c && d->lz.step == c) d->lz.step = nullptr;
    }
    Batch(const Batch&) = delete;
    Batch& operator=(const Batch&) = delete;
    int colcfg() const { return TC | CV << 8; }
    void set_col(int cfg) {
        TC = cfg & 0xff;
        CV = cfg >> 8;
    }
    Batch(ssa_ctx* c, hipStream_t s) : ctx(c), st(s) {}

    int upload_descs() {
        hops.clear(); hlz.clear(); hres.clear(); hruns.clear();
        for (auto* d : ds) {
            hops.push_back(d->op);
            hlz.push_back(d->lz);
            hres.push_back(d->rs);
            hruns.push_back(d->rn);
        }
        int rc;
        if ((rc = dops.put(hops, st))) return rc;
        if ((rc = dlz.put(hlz, st))) return rc;
        if ((rc = dres.put(hres, st))) return rc;
        if ((rc = druns.put(hruns, st))) return rc;
        return SSA_OK;
    }
    const OpDesc* ops() const { return dops.as<OpDesc>(); }
    const LzDesc* lzs() const { return dlz.as<LzDesc>(); }
    const ResDesc* res() const { return dres.as<ResDesc>(); }
    const Runs* runs() const { return druns.as<Runs>(); }
};

// HIP-event span around one launch when its kernel class is being timed
// (kind NULL: never); bytes() gives the launch's algorithmic bytes and is
// called only for a recorded launch.
struct ProfSpan {
    ssa_ctx* c;
    hipStream_t st;
    bool on = false;
    int e0 = -1;
    int e1 = -1;
    template <typename F>
    ProfSpan(ssa_ctx* ctx, const char* kind, hipStream_t s, F bytes_fn) : c(ctx), st(s) {
        if (!kind) return;
        std::lock_guard<std::mutex> g(c->mu);
        if (c->prof_kinds.empty()) return;
        const int k = c->prof_index(kind);
        if (k < 0) return;
        if (c->prof_seen[k]++ % c->prof_every) return;   // not in the sample
        // both events are taken now, so spans of concurrent threads never share one
        e0 = c->prof_event();
        e1 = e0 >= 0 ? c->prof_event() : -1;
        if (e1 < 0) return;
        (void)hipEventRecord(c->ev_pool[e0], st);
        c->spans.push_back({e0, e1, k, bytes_fn()});
        on = true;
    }
    ~ProfSpan() {
        if (!on) return;
        std::lock_guard<std::mutex> g(c->mu);
        (void)hipEventRecord(c->ev_pool[e1], st);
    }
};

// Algorithmic bytes of one column launch: every tile reads its input rows
// and the spectrum columns and writes its output rows.
double col_bytes(const Batch& b, const ItemList& L, int nin, int nout) {
    double tot = 0.0;
    for (const Item& it : L.h) {
        const auto* d = b.ds[it.inst];
        const int tc = std::min(b.TC, d->P - it.idx * b.TC);
        tot += (double)tc * (col_rows(d->op, nin) + col_rows(d->op, nout) + d->MA) * d->celem();
    }
    return tot;
}

// Algorithmic bytes of one row launch: rows x (P complex) in and/or out plus
// the compact vectors it reads or writes (vec(d) bytes per instance).  cin =
// -1: every item reads all A rows of its instance.
template <typename F>
double row_bytes(const Batch& b, const ItemList& L, int cin, int cout, F vec) {
    double tot = 0.0;
    for (const Item& it : L.h) {
        if (it.aux < 0) continue;   // padding
        const auto* d = b.ds[it.inst];
        const int ci = cin < 0 ? d->A : cin;
        tot += (double)std::max(it.aux, 1) * d->P * d->celem() * (ci + cout);
    }
    std::vector<char> seen(b.ds.size(), 0);
    for (const Item& it : L.h)
        if (!seen[it.inst]) { seen[it.inst] = 1; tot += vec(b.ds[it.inst]); }
    return tot;
}

// The LDS row kernels of the smallest size class run several items per
// workgroup and stage one twiddle table per workgroup.  In a batch whose row
// transform lengths differ, every (instance, component) run of a row item
// list is padded to a whole number of workgroups with copies of its last
// item marked aux = -1 (computed, never written), so no workgroup mixes
// lengths.
bool mixed_rows(const Batch& b) {
    if (row_slots(b.cls) <= 1) return false;
    for (auto* d : b.ds)
        if (d->nh != b.ds[0]->nh) return true;
    return false;
}

void slot_pad(const Batch& b, ItemList& L) {
    if (!mixed_rows(b)) return;
    const size_t s = (size_t)row_slots(b.cls);
    std::vector<Item> out;
    out.reserve(L.h.size() + L.h.size() / 4 + s);
    for (size_t k = 0; k < L.h.size();) {
        size_t e = k;
        while (e < L.h.size() && L.h[e].inst == L.h[k].inst && L.h[e].comp == L.h[k].comp) ++e;
        out.insert(out.end(), L.h.begin() + k, L.h.begin() + e);
        Item pad = L.h[e - 1];
        pad.aux = -1;
        while (out.size() % s) out.push_back(pad);
        k = e;
    }
    L.h.swap(out);
}

// Column-pass row code of a side's set (0: window box rows, 1: origin box rows).
inline int side_rows(int side) { return side == 0 ? ROWS_S0 : ROWS_S1; }

// rows [0, nrows) of every listed instance, optional component range; with
// group > 1 one item per group of rows (first row, row count in aux); with
// keep, only the (instance, component) pairs it accepts
void rows_items(ItemList& L, const std::vector<int>& inst, std::function<int(int)> nrows, int ncomp = 1,
                const std::vector<int>* comps = nullptr, int group = 1,
                std::function<bool(int, int)> keep = nullptr) {
    L.h.clear();
    for (int c = 0; c < ncomp; ++c)
        for (int i : inst) {
            const int nr = nrows(i);
            const int comp = comps ? (*comps)[c] : c;
            if (keep && !keep(i, comp)) continue;
            for (int a = 0; a < nr; a += group) L.h.push_back(Item{i, a, comp, std::min(group, nr - a)});
        }
}

// Short side of the bidiagonalisation: the window set unless the origin box
// is smaller (the row family always works on the window side).  It depends
// on sizes known before the origin count, so batching can use it.
int plan_side(const ssa_decomp* d) { return d->rowfam || d->L <= (long)d->KA * d->KB ? 0 : 1; }

void choose_side(ssa_decomp* d) {
    d->side = plan_side(d);
    d->nshort = d->side == 0 ? d->L : d->K;
    d->nlong = d->side == 0 ? d->K : d->L;
}

// Shape setup, origin counts, weights and the image spectrum.
int run_setup(Batch& b) {
    const int ni = (int)b.ds.size();
    hipStream_t st = b.st;
    std::vector<int> all(ni);
    for (int i = 0; i < ni; ++i) all[i] = i;
    int rc;
    if ((rc = b.upload_descs())) return rc;
    // pointer tables
    std::vector<const double*> px(ni);
    std::vector<const uint8_t*> pm(ni);
    std::vector<uint8_t*> pn(ni), pk(ni);
    std::vector<double*> pxc(ni), pw(ni);
    std::vector<int*> pnp(ni), pkp(ni), pkc(ni), pkr(ni);
    std::vector<int> nr(ni);
    for (int i = 0; i < ni; ++i) {
        auto* d = b.ds[i];
        px[i] = d->x; pm[i] = d->mask; pn[i] = d->nset; pk[i] = d->kmask;
        pxc[i] = d->xc; pw[i] = d->W; pnp[i] = d->npref; pkp[i] = d->kpref;
        pkc[i] = d->kcount; pkr[i] = d->krow; nr[i] = d->KA;
    }
    std::vector<long> tot(ni, 0);
    // windows without mask (full box) take the sliding column sums for the
    // origin counts and the weights; masked windows sum over window runs
    std::vector<int> full, masked;
    for (int i = 0; i < ni; ++i) (b.ds[i]->L == (long)b.ds[i]->LA * b.ds[i]->LB ? full : masked).push_back(i);
    ItemList rowsA, rowsK, wrows, kcols, wcols;
    rows_items(rowsA, all, [&](int i) { return b.ds[i]->A; });
    rows_items(rowsK, all, [&](int i) { return b.ds[i]->KA; });
    rows_items(wrows, masked, [&](int i) { return b.ds[i]->A; });
    for (int i : full) {
        for (int c = 0; c < (b.ds[i]->KB + 255) / 256; ++c) kcols.h.push_back(Item{i, c, 0, 0});
        for (int c = 0; c < (b.ds[i]->B + 255) / 256; ++c) wcols.h.push_back(Item{i, c, 0, 0});
    }
    TablePack tp;
    const size_t opx = tp.add(px), opm = tp.add(pm), opn = tp.add(pn), opk = tp.add(pk), opxc = tp.add(pxc),
                 opw = tp.add(pw), opnp = tp.add(pnp), opkp = tp.add(pkp), opkc = tp.add(pkc), opkr = tp.add(pkr),
                 onr = tp.add(nr), otot = tp.add(tot), oa = tp.add(rowsA.h), ok = tp.add(rowsK.h),
                 owr = tp.add(wrows.h), okc = tp.add(kcols.h), owc = tp.add(wcols.h);
    if ((rc = tp.upload(st))) return rc;
    const Item* ia = tp.at<Item>(oa);
    const Item* ik = tp.at<Item>(ok);
    launch_shape_clean(rowsA.n(), st, b.ops(), ia, tp.at<const double*>(opx), tp.at<const uint8_t*>(opm),
                       tp.at<uint8_t*>(opn), tp.at<double*>(opxc), tp.at<int*>(opnp));
    launch_shape_vcount(kcols.n(), st, b.ops(), tp.at<Item>(okc), tp.at<const int*>(opnp), tp.at<int*>(opkp));
    launch_shape_origins(rowsK.n(), st, b.ops(), ik, b.runs(), tp.at<const int*>(opnp), tp.at<uint8_t*>(opk),
                         tp.at<int*>(opkp), tp.at<int*>(opkc));
    launch_shape_rowoff(ni, st, tp.at<const int*>(opkc), tp.at<int*>(opkr), tp.at<int>(onr), tp.at<long>(otot));
    launch_shape_weights(wrows.n(), st, b.ops(), tp.at<Item>(owr), b.runs(), tp.at<const int*>(opkp),
                         tp.at<double*>(opw));
    launch_shape_weights_v(wcols.n(), st, b.ops(), tp.at<Item>(owc), tp.at<const int*>(opkp), tp.at<double*>(opw));
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(tot.data(), tp.at<long>(otot), ni * sizeof(long), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int i = 0; i < ni; ++i) {
        auto* d = b.ds[i];
        d->K = tot[i];
        d->op.S[1].count = d->K;
        // every origin of the box is in K: the row visits skip the mask
        if (d->K == (long)d->KA * d->KB) d->op.S[1].mask = nullptr;
        if (d->K == 0) d->status = fail(SSA_EEMPTY, "no window position fits inside the array");
        else if (d->r >= std::min(d->L, d->K)) d->status = fail(SSA_ERANK, "r must be < min(L, K)");
    }
    return SSA_OK;
}

// Column autotuner: the first batch of a (precision, column length) times
// the column product passes of one bidiagonalisation step (on the batch's
// own spectrum; the buffers they write are scratch at this point) with every
// compiled configuration (tile width x kernel variant) and keeps the fastest
// for the context.  The spectrum pass itself is idempotent.  SHSSA_COL_TILE
// forces a configuration (tile + 256 * variant); SHSSA_TUNE_LOG prints the
// timings.
int tune_col_tile(Batch& b) {
    std::lock_guard<std::mutex> tune_lock(b.ctx->tune_mu);
    const auto* d0 = b.ds[0];
    const auto key = std::make_pair((int)b.f64, d0->MA);
    if (const char* e = std::getenv("SHSSA_COL_TILE")) {
        const int cfg = std::atoi(e);
        if (col_tile_ok(b.f64, d0->MA, cfg)) {
            b.set_col(cfg);
            return SSA_OK;
        }
    }
    auto it = b.ctx->col_tc.find(key);
    if (it != b.ctx->col_tc.end() && col_tile_ok(b.f64, d0->MA, it->second)) {
        b.set_col(it->second);
        return SSA_OK;
    }
    hipStream_t st = b.st;
    const int ni = (int)b.ds.size();
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    float best = 1e30f;
    int best_tc = col_tile(b.f64);
    const int cands32[] = {4, 8, 16, 4 | 256, 8 | 256, 16 | 256}, cands64[] = {2, 4, 2 | 256, 4 | 256};
    const int* cands = b.f64 ? cands64 : cands32;
    const int nc = b.f64 ? 4 : 6;
    int rc = SSA_OK;
    for (int k = 0; k < nc && rc == SSA_OK; ++k) {
        const int cfg = cands[k], tc = cfg & 0xff;
        if (!col_tile_ok(b.f64, d0->MA, cfg)) continue;
        ItemList cols;
        for (int i = 0; i < ni; ++i)
            for (int t = 0; t < (b.ds[i]->P + tc - 1) / tc; ++t) cols.h.push_back(Item{i, t, 0, 0});
        if ((rc = cols.upload(st))) break;
        // the spectrum pass (also the warm-up), then the two product passes
        // of a bidiagonalisation step, timed
        launch_col(b.f64, cols.n(), st, b.ops(), b.res(), cols.ptr(), ColArgs{COL_SPEC, ROWS_ALL, 0}, d0->MA, cfg);
        const ColArgs fw{COL_CORR, side_rows(d0->side), side_rows(1 - d0->side)};
        const ColArgs bw{COL_CORR, side_rows(1 - d0->side), side_rows(d0->side)};
        (void)hipEventRecord(e0, st);
        for (int rep = 0; rep < 4; ++rep) {
            launch_col(b.f64, cols.n(), st, b.ops(), b.res(), cols.ptr(), fw, b.ds[0]->MA, cfg);
            launch_col(b.f64, cols.n(), st, b.ops(), b.res(), cols.ptr(), bw, b.ds[0]->MA, cfg);
        }
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) { rc = fail(SSA_EDEVICE, "tuning"); break; }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (std::getenv("SHSSA_TUNE_LOG"))
            std::fprintf(stderr, "column tuner: MA %d f64 %d tile %d variant %d: %.3f ms\n", d0->MA, (int)b.f64, tc,
                         cfg >> 8, ms / 8);
        // the default is kept unless another configuration is clearly (5%) faster
        if (cfg == col_tile(b.f64)) ms *= 0.95f;
        if (ms < best) { best = ms; best_tc = cfg; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    b.ctx->col_tc[key] = best_tc;
    b.ctx->tune_save("col", key.first, key.second, best_tc);
    b.set_col(best_tc);
    return SSA_OK;
}

// Allocate the operator scratch, Lanczos state and results; build the
// spectrum.  Instances with a failed status are skipped by the caller.
int run_alloc_spectrum(Batch& b) {
    hipStream_t st = b.st;
    int rc;
    if ((rc = b.dstep.put(std::vector<int>{0, 0}, st))) return rc;
    for (auto* d : b.ds) {
        const size_t ce = d->celem();
        const long xh = d->rowfam ? (long)d->A * d->ldp : (long)d->ldp * d->MA;
        d->tslot = (long)d->A * d->ldp;
        d->uslot = d->rowfam ? (long)d->P : (long)d->P * d->MA;
        const int nslot = std::max(1, d->r);
        char *xh_p, *t1, *t2, *us, *lb;
        if ((rc = d->dalloc(&xh_p, xh * ce)) || (rc = d->dalloc(&t1, d->tslot * ce * nslot)) ||
            (rc = d->dalloc(&t2, d->tslot * ce * nslot)) || (rc = d->dalloc(&us, d->uslot * ce * nslot)) ||
            (rc = d->dalloc(&lb, 2 * d->nlong * (d->f64 ? 8 : 4))))
            return rc;
        d->Xh = xh_p; d->T1 = t1; d->T2 = t2; d->Us = us; d->lbuf = lb;
        const long n = d->nshort;
        const int nblk = (int)((n + kLzRows - 1) / kLzRows);
        const long longrows = d->side == 0 ? d->KA : d->LA;
        if ((rc = d->dalloc(&d->Q, n * (kMaxBasis + 1))) || (rc = d->dalloc(&d->w, n)) ||
            (rc = d->dalloc(&d->sinv, n)) || (rc = d->dalloc(&d->hp1, (long)nblk * (kMaxBasis + 1))) ||
            (rc = d->dalloc(&d->hp2, (long)nblk * (kMaxBasis + 1))) || (rc = d->dalloc(&d->np, nblk)) ||
            (rc = d->dalloc(&d->np0, nblk)) || (rc = d->dalloc(&d->gam, 2)) ||
            (rc = d->dalloc(&d->lnp, 2 * longrows)) || (rc = d->dalloc(&d->Bm, kMaxBasis * kMaxBasis)) ||
            (rc = d->dalloc(&d->Yl, kMaxBasis * kMaxBasis)) || (rc = d->dalloc(&d->Yr, kMaxBasis * kMaxBasis)) ||
            (rc = d->dalloc(&d->sig, kMaxBasis)) || (rc = d->dalloc(&d->beta, 4)) ||
            (rc = d->dalloc(&d->perm, kMaxBasis)) || (rc = d->dalloc(&d->flag, 4)) ||
            (rc = d->dalloc(&d->Qtmp, n * kMaxBasis)) || (rc = d->dalloc(&d->U, d->L * (long)d->r)) ||
            (rc = d->dalloc(&d->V, d->K * (long)d->r)) || (rc = d->dalloc(&d->sigma, d->r)) ||
            (d->q32 && (rc = d->dalloc(&d->Q32, n * (kMaxBasis + 1)))))
            return rc;
        // descriptors
        OpDesc& o = d->op;
        o.Xh = d->Xh; o.T1 = d->T1; o.T2 = d->T2; o.Us = d->Us;
        o.tslot = d->tslot; o.uslot = d->uslot;
        if (!make_plan(d->nh, o.prow)) return fail(SSA_EINVAL, "row transform length not smooth");
        if ((rc = b.ctx->twiddles(d->nh, d->f64, false, &o.prow.tw))) return rc;
        if ((rc = b.ctx->twiddles(d->nh, d->f64, true, &o.prow.twr))) return rc;
        if (!d->rowfam) {
            if (!make_plan(d->MA, o.pcol)) return fail(SSA_EINVAL, "column transform length not smooth");
            if ((rc = b.ctx->twiddles(d->MA, d->f64, false, &o.pcol.tw))) return rc;
            o.pcol.twr = nullptr;
        }
        LzDesc& z = d->lz;
        z.seed = d->seed;
        z.step = b.dstep.as<int>();
        z.side = d->side;
        z.active = 1;
        z.r = d->r;
        z.tol = 0.1 * (d->f64 ? 1e-10 : 1e-5);
        z.eps = d->f64 ? 1e-12 : 1e-5;
        z.n = n;
        z.nl = d->nlong;
        z.Q = d->Q; z.w = d->w; z.sin = d->sinv; z.hp1 = d->hp1; z.hp2 = d->hp2; z.np = d->np; z.np0 = d->np0;
        z.lbuf[0] = d->lbuf;
        z.lbuf[1] = static_cast<char*>(d->lbuf) + d->nlong * (d->f64 ? 8 : 4);
        z.lnp[0] = d->lnp;
        z.lnp[1] = d->lnp + longrows;
        z.gam = d->gam;
        z.lwords = 2 * d->nlong * (d->f64 ? 2 : 1);   // zeroed by the start kernel
        z.lrows = (int)longrows;
        z.Bm = d->Bm; z.Yl = d->Yl; z.Yr = d->Yr; z.sig = d->sig; z.perm = d->perm;
        z.beta = d->beta; z.flag = d->flag; z.Qtmp = d->Qtmp;
        z.Q32 = d->q32 ? d->Q32 : nullptr;
        z.nblk = nblk;
        ResDesc& s = d->rs;
        s.r = d->r;
        s.U = d->U; s.V = d->V; s.sigma = d->sigma;
    }
    if ((rc = b.upload_descs())) return rc;
    // spectrum
    const int ni = (int)b.ds.size();
    std::vector<int> all(ni);
    for (int i = 0; i < ni; ++i) all[i] = i;
    ItemList rowsA;
    rows_items(rowsA, all, [&](int i) { return b.ds[i]->A; });
    slot_pad(b, rowsA);
    if ((rc = rowsA.upload(st))) return rc;
    const auto* d0 = b.ds[0];
    if (d0->rowfam) {
        // row spectra scaled by 1/MB straight into each instance's Xh
        RowInArgs a{IN_DENSE, 0, 0, DEST_XH, -1.0, 0};   // each instance's spec_scale
        launch_row_in(b.f64, b.cls, rowsA.n(), st, b.ops(), b.lzs(), b.res(), rowsA.ptr(), a);
    } else {
        RowInArgs a{IN_DENSE, 0, 0, DEST_T1, 1.0, 0};
        launch_row_in(b.f64, b.cls, rowsA.n(), st, b.ops(), b.lzs(), b.res(), rowsA.ptr(), a);
        if ((rc = tune_col_tile(b))) return rc;
        ItemList cols;
        for (int i = 0; i < ni; ++i)
            for (int t = 0; t < (b.ds[i]->P + b.TC - 1) / b.TC; ++t) cols.h.push_back(Item{i, t, 0, 0});
        if ((rc = cols.upload(st))) return rc;
        launch_col(b.f64, cols.n(), st, b.ops(), b.res(), cols.ptr(), ColArgs{COL_SPEC, ROWS_ALL, 0}, d0->MA, b.colcfg());
    }
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipGetLastError());
    return SSA_OK;
}

// One application of the bidiagonalisation step j (products and
// reorthogonalisation) for the listed instances.
struct StepLists {
    ItemList rin, cols, rmid, rout, lzb, inst;
};

void build_step_lists(Batch& b, const std::vector<int>& act, StepLists& S) {
    const auto* d0 = b.ds[0];
    const int s = d0->side;
    if (d0->rowfam) {
        rows_items(S.rin, act, [&](int) { return 1; }, 1, nullptr, row_group(b.cls, false));
        rows_items(S.rmid, act, [&](int i) { return b.ds[i]->A; });
        rows_items(S.rout, act, [&](int) { return 1; });
        S.cols.h.clear();
    } else {
        rows_items(S.rin, act, [&](int i) { return b.ds[i]->op.S[s].boxA; }, 1, nullptr, row_group(b.cls, false));
        rows_items(S.rmid, act, [&](int i) { return b.ds[i]->op.S[1 - s].boxA; }, 1, nullptr,
                   row_group(b.cls, false));
        rows_items(S.rout, act, [&](int i) { return b.ds[i]->op.S[s].boxA; }, 1, nullptr, row_group(b.cls, false));
        S.cols.h.clear();
        for (int i : act)
            for (int t = 0; t < (b.ds[i]->P + b.TC - 1) / b.TC; ++t) S.cols.h.push_back(Item{i, t, 0, 0});
    }
    slot_pad(b, S.rin);
    slot_pad(b, S.rmid);
    slot_pad(b, S.rout);
    S.lzb.h.clear();
    S.inst.h.clear();
    for (int i : act) {
        for (int k = 0; k < b.ds[i]->lz.nblk; ++k) S.lzb.h.push_back(Item{i, k, 0, 0});
        S.inst.h.push_back(Item{i, 0, 0, 0});
    }
}

int upload_step_lists(StepLists& S, hipStream_t st) {
    return upload_lists({&S.rin, &S.cols, &S.rmid, &S.rout, &S.lzb, &S.inst}, st);
}

// j = kStepDev (with mode IN_LZ_STEP): the step comes from the batch's
// step counter (a step captured once and replayed).  prof = false: no
// timing spans (a captured step).
void launch_step(Batch& b, StepLists& S, int j, int jstart, int mode, bool prof = true) {
    hipStream_t st = b.st;
    const auto* d0 = b.ds[0];
    const int s = d0->side;
    // compact vector bytes per instance: short side FP64, long side in the operator precision
    const auto vs = [&](const ssa_decomp* d) { return 8.0 * d->nshort; };
    const auto vl2 = [&](const ssa_decomp* d) { return 2.0 * (d->f64 ? 8.0 : 4.0) * d->nlong; };
    const auto vs2 = [&](const ssa_decomp* d) { return 16.0 * d->nshort; };
    if (d0->rowfam) {
        {
            ProfSpan p(b.ctx, prof ? "row_in" : nullptr, st, [&] { return row_bytes(b, S.rin, 0, 1, vs); });
            launch_row_in(b.f64, b.cls, S.rin.n(), st, b.ops(), b.lzs(), b.res(), S.rin.ptr(),
                          RowInArgs{mode, 0, j, DEST_T1, 1.0, 0});
        }
        {
            ProfSpan p(b.ctx, prof ? "rowfam_mid" : nullptr, st, [&] { return row_bytes(b, S.rmid, 3, 1, vl2); });
            launch_rowfam_mid(b.f64, b.cls, S.rmid.n(), st, b.ops(), b.lzs(), b.res(), S.rmid.ptr(),
                              RowFamArgs{OUT_NONE, 1, 1, j, jstart});
        }
        {
            ProfSpan p(b.ctx, prof ? "rowfam_out" : nullptr, st, [&] { return row_bytes(b, S.rout, -1, 0, vs2); });
            launch_rowfam_out(b.f64, b.cls, S.rout.n(), st, b.ops(), b.lzs(), S.rout.ptr(),
                              RowOutArgs{OUT_LZ, 0, 1.0, 0, j, jstart});
        }
    } else {
        const int nin = side_rows(s), nmid = side_rows(1 - s);
        {
            ProfSpan p(b.ctx, prof ? "row_in" : nullptr, st, [&] { return row_bytes(b, S.rin, 0, 1, vs); });
            launch_row_in(b.f64, b.cls, S.rin.n(), st, b.ops(), b.lzs(), b.res(), S.rin.ptr(),
                          RowInArgs{mode, s, j, DEST_T1, 1.0, 0});
        }
        {
            ProfSpan p(b.ctx, prof ? "col" : nullptr, st, [&] { return col_bytes(b, S.cols, nin, nmid); });
            launch_col(b.f64, S.cols.n(), st, b.ops(), b.res(), S.cols.ptr(),
                       ColArgs{COL_CORR, nin, nmid}, d0->MA, b.colcfg());
        }
        {
            ProfSpan p(b.ctx, prof ? "row_mid" : nullptr, st, [&] { return row_bytes(b, S.rmid, 1, 1, vl2); });
            launch_row_mid(b.f64, b.cls, S.rmid.n(), st, b.ops(), b.lzs(), b.res(), S.rmid.ptr(),
                           RowMidArgs{1 - s, OUT_NONE, 1.0, 0, 1, 1, j, jstart});
        }
        {
            ProfSpan p(b.ctx, prof ? "col" : nullptr, st, [&] { return col_bytes(b, S.cols, nmid, nin); });
            launch_col(b.f64, S.cols.n(), st, b.ops(), b.res(), S.cols.ptr(),
                       ColArgs{COL_CORR, nmid, nin}, d0->MA, b.colcfg());
        }
        {
            ProfSpan p(b.ctx, prof ? "row_out" : nullptr, st, [&] { return row_bytes(b, S.rout, 1, 0, vs2); });
            launch_row_out(b.f64, b.cls, S.rout.n(), st, b.ops(), b.lzs(), b.res(), S.rout.ptr(),
                           RowOutArgs{OUT_LZ, s, 1.0, 0, j, jstart});
        }
    }
    const int ncols = j == kStepDev ? -1 : j + 1;   // -1: from the step counter
    const auto qb = [&] {
        double t = 0.0;
        for (const Item& it : S.inst.h) t += 8.0 * b.ds[it.inst]->nshort * ncols;
        return t;
    };
    {
        ProfSpan p(b.ctx, prof ? "lz_proj" : nullptr, st, qb);
        launch_lz_proj(S.lzb.n(), st, b.lzs(), S.lzb.ptr(), ncols);
    }
    {
        ProfSpan p(b.ctx, prof ? "lz_update" : nullptr, st, qb);
        launch_lz_update(S.lzb.n(), st, b.lzs(), S.lzb.ptr(), ncols, 1, 0);
    }
    // second Gram-Schmidt pass for FP64 instances, skipped on the device
    // when not needed.  FP32-product instances make one FP64 pass: it
    // leaves eps |w_before| / |w_after| of the basis in w, below the
    // products' own 1e-7 unless the pass cancels w by nine orders (where
    // the breakdown test takes over).  With SSA_FP32_BASIS32 the pass reads
    // the FP32 copy of the basis, whose rounding (about 1e-7) then bounds
    // the orthogonality.
    if (b.f64) {
        launch_lz_proj2(S.lzb.n(), st, b.lzs(), S.lzb.ptr(), ncols, 0);
        launch_lz_update(S.lzb.n(), st, b.lzs(), S.lzb.ptr(), ncols, 2, 0);
    }
}

// Basis size m and restart size kk of the thick-restart bidiagonalisation.
// The basis holds r plus min(r + 20, 50) further vectors (at most
// kMaxBasis and the short side): past about 50 extra vectors each cycle's
// longer reorthogonalisations and larger small SVD cost more than its fewer
// restarts save (64-image batches of 512 x 512 with a 64 x 64 window).  A
// restart keeps kk = m - m / q Ritz vectors, q >= 2 the smallest divisor of
// m (m rounded down to a multiple of q) that leaves kk >= r: every cycle
// after the first adds c = m / q vectors and the first one, from a start
// vector, adds m = q c.  So an instance that starts at a cycle boundary of
// a running batch meets all its later boundaries, with the steps it would
// take alone (continuous batching).  For r <= 50 this keeps half the
// basis, r + 10 Ritz vectors at r = 30, where keeping a quarter of the
// extra vectors (42) measured the same within noise.
int basis_size(long nshort, int r) {
    int m0 = std::min(2 * r + 20, r + 50);
    if (const char* e = std::getenv("SHSSA_BASIS")) m0 = std::max(r + 2, std::atoi(e));   // experiments
    m0 = std::min(m0, kMaxBasis);
    if (nshort <= m0) m0 = (int)nshort;
    for (int q = 2; q <= m0; ++q) {
        const int m = m0 - m0 % q, kk = m - m / q;
        if (kk >= r && kk < m) return m;
    }
    return m0;
}

// Ritz vectors kept by a restart of a basis of size m (see basis_size).
int restart_keep(int m, int r) {
    for (int q = 2; q <= m; ++q)
        if (m % q == 0 && m - m / q >= r && m - m / q < m) return m - m / q;
    return std::max(r, m - 1);
}

// Bidiagonalisation steps (all their launches, each step read from the
// batch's counter, which the last launch of a step advances) captured as a
// HIP graph and replayed while the batch's item lists stay the same: one
// graph launch instead of ten kernel launches per step.  SHSSA_GRAPHS=n
// (n >= 1 steps per graph) turns it on; by default the kernels are launched
// directly, which measured as fast or faster here (64 images of 512 x 512:
// 73.5 ms per batch direct, 75-77 ms with graphs of 1 to 45 steps).  A
// context on the null stream (which cannot be captured) launches directly.
struct StepGraph {
    hipStream_t st = nullptr;
    hipGraphExec_t exec = nullptr;
    bool on = false;
    int steps = 1;   // steps per captured graph
    explicit StepGraph(hipStream_t s) : st(s) {
        const char* e = std::getenv("SHSSA_GRAPHS");
        on = st != nullptr && e && std::atoi(e) > 0;
        if (on) steps = std::max(1, std::atoi(e));
    }
    // caller has waited for the stream (replays done)
    void reset() {
        if (exec) (void)hipGraphExecDestroy(exec);
        exec = nullptr;
    }
    ~StepGraph() {
        if (exec) (void)hipStreamSynchronize(st);
        reset();
    }
    // capture the step; on failure graphs are switched off for the batch
    bool capture(Batch& b, StepLists& S) {
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return on = false;
        for (int k = 0; k < steps; ++k) {
            launch_step(b, S, kStepDev, kStepDev, IN_LZ_STEP, false);
            launch_step_next(st, b.dstep.as<int>());
        }
        const hipError_t e1 = hipStreamEndCapture(st, &g);
        const hipError_t e2 = e1 == hipSuccess ? hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) : e1;
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        if (e2 != hipSuccess) {
            exec = nullptr;
            return on = false;
        }
        return true;
    }
};

// Kernel classes of one step and their launches (for the timing sample).
std::vector<std::pair<const char*, int>> step_classes(bool rowfam) {
    if (rowfam) return {{"row_in", 1}, {"rowfam_mid", 1}, {"rowfam_out", 1}, {"lz_proj", 1}, {"lz_update", 1}};
    return {{"row_in", 1}, {"col", 2}, {"row_mid", 1}, {"row_out", 1}, {"lz_proj", 1}, {"lz_update", 1}};
}

// Thick restart of the instances in cont from the last cycle (basis m):
// the k leading Ritz vectors are kept; the instances in fresh restart from
// a random vector orthogonal to them instead of the residual.
int launch_restart(Batch& b, const std::vector<int>& cont, const std::vector<int>& fresh, int m, int kk,
                   int cycle) {
    hipStream_t st = b.st;
    int rc;
    ItemList R, Z, F;
    std::vector<char> isfresh(b.ds.size(), 0);
    for (int i : fresh) isfresh[i] = 1;
    for (int i : cont) {
        const long n = b.ds[i]->nshort;
        for (long rb = 0; rb < (n + 63) / 64; ++rb)
            for (int cb = 0; cb < (kk + 31) / 32; ++cb) R.h.push_back(Item{i, (int)rb, 0, cb});
        for (int k = 0; k < b.ds[i]->lz.nblk; ++k) (isfresh[i] ? F : Z).h.push_back(Item{i, k, 0, 0});
    }
    if ((rc = upload_lists({&R, &Z, &F}, st))) return rc;
    {
        ProfSpan p(b.ctx, "lz_ritz", st, [&] {
            double f = 0.0;
            for (int i : cont) f += 2.0 * b.ds[i]->nshort * m * kk;
            return f;
        });
        launch_lz_ritz(R.n(), st, b.lzs(), R.ptr(), m, kk, nullptr);
    }
    launch_lz_restart(Z.n(), st, b.lzs(), Z.ptr(), m, kk);
    if (F.n() > 0) {
        launch_lz_restart_random(F.n(), st, b.lzs(), F.ptr(), kk, 7919ULL * cycle);   // ^ own seed
        launch_lz_proj(F.n(), st, b.lzs(), F.ptr(), kk);
        launch_lz_update(F.n(), st, b.lzs(), F.ptr(), kk, 1, 1);
        launch_lz_proj2(F.n(), st, b.lzs(), F.ptr(), kk, 1);
        launch_lz_update(F.n(), st, b.lzs(), F.ptr(), kk, 2, 1);
    }
    return SSA_OK;
}

// resume_m > 0: continue a finished bidiagonalisation whose last cycle had
// a basis of resume_m vectors (its Ritz vectors and residual are still in
// the instances' state): a thick restart keeps its leading Ritz vectors and
// the cycles go on with the basis and restart size of the instances' r.
// resume_fresh: the last cycle's residual is no direction to continue in
// (the Krylov space was exhausted, or the basis was the whole short side):
// a random vector orthogonal to the kept Ritz vectors replaces it.
int run_lanczos(Batch& b, int max_steps, const std::function<int()>& overlap = nullptr, int resume_m = 0,
                bool resume_fresh = false) {
    hipStream_t st = b.st;
    const int ni = (int)b.ds.size();
    int rc;
    // every instance of a batch has the same basis size and restart size
    // (they differ in r only where the basis is clipped)
    const int m = basis_size(b.ds[0]->nshort, b.ds[0]->r);
    const int kk = restart_keep(m, b.ds[0]->r);
    int rmax = 0;
    for (auto* d : b.ds) rmax = std::max(rmax, d->r);
    // every cycle keeps kk >= r Ritz vectors and adds m - kk > 0 new ones
    if (!(rmax <= kk && kk < m && m <= kMaxBasis))
        return fail(SSA_ERANK, "rank leaves no room in the Lanczos basis");
    std::vector<int> act(ni);
    for (int i = 0; i < ni; ++i) act[i] = i;
    std::vector<int> steps(ni, 0), restarts(ni, 0);
    StepLists S;
    build_step_lists(b, act, S);
    if ((rc = upload_step_lists(S, st))) return rc;
    int jstart = 0;
    if (resume_m > 0) {
        const int k0 = std::min(kk, resume_m);
        if ((rc = launch_restart(b, act, resume_fresh ? act : std::vector<int>{}, resume_m, k0, 0))) return rc;
        jstart = k0;
    } else {
        launch_lz_start(S.lzb.n(), st, b.lzs(), S.lzb.ptr(), 0ULL);   // each instance's own seed
    }
    std::vector<int> flags(4 * ni);
    std::vector<double> betas(2 * ni);
    std::vector<int> bdrest(ni, 0);
    int cycle = 0;
    for (auto* d : b.ds) d->st.basis = m;
    StepGraph G(st);
    const auto classes = step_classes(b.ds[0]->rowfam);
    while (!act.empty()) {
        if (G.on) {
            const int ctr[2] = {jstart, jstart};
            if ((rc = b.ctx->upload(b.dstep.p, ctr, sizeof(ctr), st))) return rc;
        }
        for (int j = jstart; j < m; ++j) {
            if (G.on && j + G.steps <= m && !b.ctx->prof_take_step(classes, G.steps) &&
                (G.exec || G.capture(b, S))) {
                HIPCHK(hipGraphLaunch(G.exec, st));
                j += G.steps - 1;
                continue;
            }
            const int mode = (j == jstart && jstart > 0) ? IN_LZ_SIN : IN_LZ_NORM;
            launch_step(b, S, j, jstart, mode);
            if (G.on) launch_step_next(st, b.dstep.as<int>());
        }
        launch_lz_normalize(S.lzb.n(), st, b.lzs(), S.lzb.ptr(), m);
        {
            ProfSpan p(b.ctx, "lz_svd", st, [] { return 0.0; });
            launch_lz_svd(S.inst.n(), st, b.lzs(), S.inst.ptr(), m, 40);
        }
        HIPCHK(hipGetLastError());
        if (cycle == 0 && overlap && (rc = overlap())) return rc;   // host work while the cycle runs
        {
            // one gather kernel and one copy into pinned memory for the batch
            const size_t fb = (size_t)ni * 4 * sizeof(int), bb = (size_t)ni * 2 * sizeof(double);
            if (!b.dflag.p || b.dflag.cap < fb + bb) {
                std::vector<char> z(fb + bb, 0);
                if ((rc = b.dflag.put(z, st))) return rc;
            }
            char* dv = b.dflag.as<char>();
            launch_gather_flags(ni, st, b.lzs(), reinterpret_cast<int*>(dv), reinterpret_cast<double*>(dv + fb));
            void* hb = nullptr;
            if ((rc = b.ctx->readback_buf(st, fb + bb, &hb))) return rc;
            HIPCHK(hipMemcpyAsync(hb, dv, fb + bb, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            std::memcpy(flags.data(), hb, fb);
            std::memcpy(betas.data(), static_cast<char*>(hb) + fb, bb);
        }
        ++cycle;
        if (std::getenv("SHSSA_DEBUG")) {
            for (int i : act) {
                auto* d = b.ds[i];
                std::vector<double> Bh(kMaxBasis * kMaxBasis), sg(m), bt(4);
                (void)hipMemcpy(Bh.data(), d->Bm, Bh.size() * 8, hipMemcpyDeviceToHost);
                (void)hipMemcpy(sg.data(), d->sig, m * 8, hipMemcpyDeviceToHost);
                (void)hipMemcpy(bt.data(), d->beta, 4 * 8, hipMemcpyDeviceToHost);
                std::fprintf(stderr, "cycle %d inst %d flags %d %d %d %d beta %g %g %g %g eps %g\n", cycle, i,
                             flags[4 * i], flags[4 * i + 1], flags[4 * i + 2], flags[4 * i + 3], bt[0], bt[1], bt[2],
                             bt[3], d->lz.eps);
                std::fprintf(stderr, "  diag:");
                for (int k = 0; k < std::min(m, 8); ++k) std::fprintf(stderr, " %g", Bh[(size_t)k * kMaxBasis + k]);
                std::fprintf(stderr, "\n  sub:");
                for (int k = 0; k < std::min(m, 8); ++k) std::fprintf(stderr, " %g", Bh[(size_t)k * kMaxBasis + k + 1]);
                std::fprintf(stderr, "\n  sig:");
                for (int k = 0; k < std::min(m, 6); ++k) std::fprintf(stderr, " %g", sg[k]);
                std::fprintf(stderr, "\n");
            }
        }
        // Per instance: converged -> done; breakdown (the Krylov space of the
        // start vector is exhausted) -> restart from a random vector orthogonal
        // to the kept Ritz vectors, at most twice, then done; otherwise a thick
        // restart, up to the step limit.
        std::vector<int> done, cont, fresh;
        for (int i : act) {
            steps[i] += m - jstart;
            b.ds[i]->st.svd_sweeps += flags[4 * i + 1];
            const bool ok = flags[4 * i] != 0;
            const bool bd = flags[4 * i + 2] != 0;
            auto* d = b.ds[i];
            if (bd && bdrest[i] < 2 && steps[i] < max_steps) {
                bdrest[i]++;
                restarts[i]++;
                fresh.push_back(i);
                cont.push_back(i);
                continue;
            }
            if (ok || bd || steps[i] >= max_steps) {
                done.push_back(i);
                d->st.converged = ok || bd;
                d->st.steps = steps[i];
                d->st.restarts = restarts[i];
                d->st.max_resid = betas[2 * i + 1];
                if (!(ok || bd)) d->status = fail(SSA_ENOCONV, "bidiagonalisation reached its step limit");
            } else {
                cont.push_back(i);
                restarts[i]++;
            }
        }
        if (!done.empty()) {
            // Ritz vectors and singular values of the finished instances
            std::vector<double*> outs(ni, nullptr);
            for (int i : done) outs[i] = b.ds[i]->side == 0 ? b.ds[i]->U : b.ds[i]->V;
            DevVec douts;
            if ((rc = douts.put(outs, st))) return rc;
            ItemList R, I;
            for (int i : done) {
                const long n = b.ds[i]->nshort;
                for (long rb = 0; rb < (n + 63) / 64; ++rb)
                    for (int cb = 0; cb < (b.ds[i]->r + 31) / 32; ++cb) R.h.push_back(Item{i, (int)rb, 0, cb});
                I.h.push_back(Item{i, 0, 0, 0});
            }
            if ((rc = upload_lists({&R, &I}, st))) return rc;
            {
                // timing class "lz_ritz" counts floating-point operations, 2 n m k per instance
                ProfSpan p(b.ctx, "lz_ritz", st, [&] {
                    double f = 0.0;
                    for (int i : done) f += 2.0 * b.ds[i]->nshort * m * b.ds[i]->r;
                    return f;
                });
                launch_lz_ritz(R.n(), st, b.lzs(), R.ptr(), m, rmax, douts.as<double*>());
            }
            launch_lz_sigma(I.n(), st, b.lzs(), b.res(), I.ptr());
            // no wait: the tables are released into the call's table cache,
            // which returns them to the pool only after the stream drains
        }
        if (cont.empty()) break;
        if ((rc = launch_restart(b, cont, fresh, m, kk, cycle))) return rc;
        if (cont.size() != act.size()) {
            // the item lists change: the captured step is rebuilt (the
            // stream has been waited for at the convergence test)
            act = cont;
            G.reset();
            build_step_lists(b, act, S);
            if ((rc = upload_step_lists(S, st))) return rc;
        }
        jstart = kk;
    }
    HIPCHK(hipGetLastError());
    return SSA_OK;
}

// Ritz vectors and singular values of instances whose bidiagonalisation is
// done (into U or V by side, and sigma).
int lanczos_outputs(Batch& b, const std::vector<int>& done, int m, int rmax) {
    hipStream_t st = b.st;
    const int ni = (int)b.ds.size();
    int rc;
    std::vector<double*> outs(ni, nullptr);
    for (int i : done) outs[i] = b.ds[i]->side == 0 ? b.ds[i]->U : b.ds[i]->V;
    DevVec douts;
    if ((rc = douts.put(outs, st))) return rc;
    ItemList R, I;
    for (int i : done) {
        const long n = b.ds[i]->nshort;
        for (long rb = 0; rb < (n + 63) / 64; ++rb)
            for (int cb = 0; cb < (b.ds[i]->r + 31) / 32; ++cb) R.h.push_back(Item{i, (int)rb, 0, cb});
        I.h.push_back(Item{i, 0, 0, 0});
    }
    if ((rc = upload_lists({&R, &I}, st))) return rc;
    {
        ProfSpan p(b.ctx, "lz_ritz", st, [&] {
            double f = 0.0;
            for (int i : done) f += 2.0 * b.ds[i]->nshort * m * b.ds[i]->r;
            return f;
        });
        launch_lz_ritz(R.n(), st, b.lzs(), R.ptr(), m, rmax, douts.as<double*>());
    }
    launch_lz_sigma(I.n(), st, b.lzs(), b.res(), I.ptr());
    return SSA_OK;
}

// Continuous batching of one kernel class: at most `slots` instances of the
// batch advance together; when some finish at a cycle boundary, waiting
// instances of the batch take their slots and begin from their start
// vectors.  Each instance keeps its own step counter [j, jstart] on the
// device, which the step kernels read, so instances at different steps
// share every launch.  With the cycle plan of basis_size and restart_keep
// all boundaries are common (a first cycle lasts q later ones), and an
// instance runs exactly the steps, restarts and reductions it would run
// alone: its results do not depend on when it joined.
int run_lanczos_cont(Batch& b, int max_steps, int slots, const std::function<int()>& overlap) {
    hipStream_t st = b.st;
    const int ni = (int)b.ds.size();
    int rc;
    const int m = basis_size(b.ds[0]->nshort, b.ds[0]->r);
    const int kk = restart_keep(m, b.ds[0]->r);
    const int c = m - kk;
    int rmax = 0;
    for (auto* d : b.ds) rmax = std::max(rmax, d->r);
    if (!(rmax <= kk && kk < m && m <= kMaxBasis) || m % c != 0)
        return fail(SSA_ERANK, "rank leaves no room in the Lanczos basis");
    // per-instance step counters; on every way out the handles point at the
    // batch's shared counter again, never at these (released on return)
    DevVec dctr;
    if ((rc = dctr.reserve((size_t)ni * 2 * sizeof(int)))) return rc;
    struct StepBack {
        Batch& b;
        ~StepBack() {
            for (auto* d : b.ds) d->lz.step = b.dstep.as<int>();
        }
    } step_back{b};
    for (int i = 0; i < ni; ++i) b.ds[i]->lz.step = dctr.as<int>() + 2 * i;
    if ((rc = b.upload_descs())) return rc;
    std::vector<int> act, pending;
    for (int i = 0; i < ni; ++i) (i < slots ? act : pending).push_back(i);
    std::vector<int> steps(ni, 0), restarts(ni, 0), jh(ni, 0), cycles(ni, 0), bdrest(ni, 0);
    std::vector<int> flags(4 * ni);
    std::vector<double> betas(2 * ni);
    for (auto* d : b.ds) d->st.basis = m;
    // start vectors and counters [0, 0] of instances entering the batch
    const auto start = [&](const std::vector<int>& who) -> int {
        ItemList Z, I;
        for (int i : who) {
            for (int k = 0; k < b.ds[i]->lz.nblk; ++k) Z.h.push_back(Item{i, k, 0, 0});
            I.h.push_back(Item{i, 0, 0, 0});
            jh[i] = 0;
        }
        int e;
        if ((e = upload_lists({&Z, &I}, st))) return e;
        launch_lz_start(Z.n(), st, b.lzs(), Z.ptr(), 0ULL);   // each instance's own seed
        launch_step_set(I.n(), st, b.lzs(), I.ptr(), 0, 0);
        return SSA_OK;
    };
    if ((rc = start(act))) return rc;
    StepLists S;
    build_step_lists(b, act, S);
    if ((rc = upload_step_lists(S, st))) return rc;
    bool first = true;
    while (!act.empty()) {
        for (int k = 0; k < c; ++k) {
            launch_step(b, S, kStepDev, kStepDev, IN_LZ_STEP);
            launch_step_next_inst(S.inst.n(), st, b.lzs(), S.inst.ptr());
        }
        HIPCHK(hipGetLastError());
        if (first && overlap && (rc = overlap())) return rc;   // host work while the steps run
        first = false;
        std::vector<int> ends, rest;
        for (int i : act) {
            jh[i] += c;
            (jh[i] == m ? ends : rest).push_back(i);
        }
        std::vector<int> done, cont, fresh;
        if (!ends.empty()) {
            ItemList N, I;
            for (int i : ends) {
                for (int k = 0; k < b.ds[i]->lz.nblk; ++k) N.h.push_back(Item{i, k, 0, 0});
                I.h.push_back(Item{i, 0, 0, 0});
            }
            if ((rc = upload_lists({&N, &I}, st))) return rc;
            launch_lz_normalize(N.n(), st, b.lzs(), N.ptr(), m);
            {
                ProfSpan p(b.ctx, "lz_svd", st, [] { return 0.0; });
                launch_lz_svd(I.n(), st, b.lzs(), I.ptr(), m, 40);
            }
            HIPCHK(hipGetLastError());
            const size_t fb = (size_t)ni * 4 * sizeof(int), bb = (size_t)ni * 2 * sizeof(double);
            if (!b.dflag.p || b.dflag.cap < fb + bb) {
                std::vector<char> z(fb + bb, 0);
                if ((rc = b.dflag.put(z, st))) return rc;
            }
            char* dv = b.dflag.as<char>();
            launch_gather_flags(ni, st, b.lzs(), reinterpret_cast<int*>(dv), reinterpret_cast<double*>(dv + fb));
            void* hb = nullptr;
            if ((rc = b.ctx->readback_buf(st, fb + bb, &hb))) return rc;
            HIPCHK(hipMemcpyAsync(hb, dv, fb + bb, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            std::memcpy(flags.data(), hb, fb);
            std::memcpy(betas.data(), static_cast<char*>(hb) + fb, bb);
            // the decisions of the lockstep loop, per instance
            for (int i : ends) {
                steps[i] += m - (cycles[i] == 0 ? 0 : kk);
                ++cycles[i];
                auto* d = b.ds[i];
                d->st.svd_sweeps += flags[4 * i + 1];
                const bool ok = flags[4 * i] != 0;
                const bool bd = flags[4 * i + 2] != 0;
                if (bd && bdrest[i] < 2 && steps[i] < max_steps) {
                    bdrest[i]++;
                    restarts[i]++;
                    fresh.push_back(i);
                    cont.push_back(i);
                    continue;
                }
                if (ok || bd || steps[i] >= max_steps) {
                    done.push_back(i);
                    d->st.converged = ok || bd;
                    d->st.steps = steps[i];
                    d->st.restarts = restarts[i];
                    d->st.max_resid = betas[2 * i + 1];
                    if (!(ok || bd)) d->status = fail(SSA_ENOCONV, "bidiagonalisation reached its step limit");
                } else {
                    cont.push_back(i);
                    restarts[i]++;
                }
            }
            if (!done.empty() && (rc = lanczos_outputs(b, done, m, rmax))) return rc;
            if (!cont.empty()) {
                // the random restart of a breakdown draws from the instance's
                // own cycle count, as in the lockstep loop
                std::map<int, std::vector<int>> by_cycle;
                std::vector<char> isf(ni, 0);
                for (int i : fresh) isf[i] = 1;
                for (int i : cont) by_cycle[isf[i] ? cycles[i] : -1].push_back(i);
                for (auto& kv : by_cycle) {
                    const std::vector<int>& grp = kv.second;
                    if ((rc = launch_restart(b, grp, kv.first < 0 ? std::vector<int>{} : grp, m, kk,
                                             kv.first < 0 ? 0 : kv.first)))
                        return rc;
                }
                ItemList I2;
                for (int i : cont) {
                    I2.h.push_back(Item{i, 0, 0, 0});
                    jh[i] = kk;
                }
                if ((rc = upload_lists({&I2}, st))) return rc;
                launch_step_set(I2.n(), st, b.lzs(), I2.ptr(), kk, kk);
            }
        }
        // the next active set: continuing and mid-cycle instances, then
        // waiting ones in the freed slots
        std::vector<int> next = rest;
        next.insert(next.end(), cont.begin(), cont.end());
        std::vector<int> joiners;
        while (!pending.empty() && (int)(next.size() + joiners.size()) < slots) {
            joiners.push_back(pending.front());
            pending.erase(pending.begin());
        }
        if (!joiners.empty() && (rc = start(joiners))) return rc;
        next.insert(next.end(), joiners.begin(), joiners.end());
        std::sort(next.begin(), next.end());
        if (next != act) {
            act = next;
            if (!act.empty()) {
                build_step_lists(b, act, S);
                if ((rc = upload_step_lists(S, st))) return rc;
            }
        }
    }
    // later launches of this batch (finish) see the batch's shared counter
    for (auto* d : b.ds) d->lz.step = b.dstep.as<int>();
    if ((rc = b.upload_descs())) return rc;
    HIPCHK(hipGetLastError());
    return SSA_OK;
}

// Bidiagonalisation steps an instance may take before it is returned with
// SSA_ENOCONV (its triplets as they stand).  SHSSA_MAX_STEPS lowers the
// limit, which lets a caller force that outcome.
int step_limit() {
    int n = 3000;
    if (const char* e = std::getenv("SHSSA_MAX_STEPS")) n = std::max(1, std::min(n, std::atoi(e)));
    return n;
}

// Item lists of the final pass (built and uploaded while the first
// bidiagonalisation cycle runs on the device).
struct FinishLists {
    ItemList rin, cols, rmid, sg;
    bool ready = false;
};

// who: the instances to finish (nullptr: all of the batch).
int finish_lists(Batch& b, FinishLists& F, const std::vector<int>* who = nullptr) {
    const int ni = (int)b.ds.size();
    std::vector<int> all(ni);
    for (int i = 0; i < ni; ++i) all[i] = i;
    if (who) all = *who;
    const auto* d0 = b.ds[0];
    int r = 0;   // components of the batch (instances may have fewer)
    for (int i : all) r = std::max(r, b.ds[i]->r);
    const int s = d0->side;
    // component c of the instances with r > c
    const auto has = [&](int i, int c) { return c < b.ds[i]->r; };
    if (d0->rowfam) {
        rows_items(F.rin, all, [&](int) { return 1; }, r, nullptr, row_group(b.cls, false), has);
        rows_items(F.rmid, all, [&](int i) { return b.ds[i]->A; }, r, nullptr, 1, has);
        F.cols.h.clear();
    } else {
        rows_items(F.rin, all, [&](int i) { return b.ds[i]->op.S[s].boxA; }, r, nullptr, row_group(b.cls, false),
                   has);
        rows_items(F.rmid, all, [&](int i) { return b.ds[i]->op.S[1 - s].boxA; }, r, nullptr,
                   row_group(b.cls, false), has);
        F.cols.h.clear();
        for (int c = 0; c < r; ++c)
            for (int i : all)
                if (has(i, c))
                    for (int t = 0; t < (b.ds[i]->P + b.TC - 1) / b.TC; ++t) F.cols.h.push_back(Item{i, t, c, 0});
    }
    slot_pad(b, F.rin);
    slot_pad(b, F.rmid);
    F.sg.h.clear();
    for (int c = 0; c < r; ++c)
        for (int i : all)
            if (has(i, c)) F.sg.h.push_back(Item{i, 0, c, 0});
    const int rc = upload_lists({&F.rin, &F.cols, &F.rmid, &F.sg}, b.st);
    F.ready = rc == SSA_OK;
    return rc;
}

// Long-side vectors of the final triplets (V = X^T U / sigma or
// U = X V / sigma), then the sign rule.
int run_finish(Batch& b, FinishLists& F, const std::vector<int>* who = nullptr) {
    hipStream_t st = b.st;
    int rc;
    if (!F.ready && (rc = finish_lists(b, F, who))) return rc;
    const auto* d0 = b.ds[0];
    const int s = d0->side;
    // short side = window side: fix the signs of U first, V = X^T U / sigma
    // then comes out with the right sign (no pass over the long vectors)
    if (s == 0) launch_sign_fix(F.sg.n(), st, b.ops(), b.res(), F.sg.ptr(), 0);
    if (d0->rowfam) {
        launch_row_in(b.f64, b.cls, F.rin.n(), st, b.ops(), b.lzs(), b.res(), F.rin.ptr(),
                      RowInArgs{IN_VEC, 0, 0, DEST_T1, 1.0, 0});
        launch_rowfam_mid(b.f64, b.cls, F.rmid.n(), st, b.ops(), b.lzs(), b.res(), F.rmid.ptr(),
                          RowFamArgs{OUT_VEC, 0, 0, 0, 0});
    } else {
        launch_row_in(b.f64, b.cls, F.rin.n(), st, b.ops(), b.lzs(), b.res(), F.rin.ptr(),
                      RowInArgs{IN_VEC, s, 0, DEST_T1, 1.0, 0});
        launch_col(b.f64, F.cols.n(), st, b.ops(), b.res(), F.cols.ptr(),
                   ColArgs{COL_CORR, side_rows(s), side_rows(1 - s)}, d0->MA, b.colcfg());
        launch_row_mid(b.f64, b.cls, F.rmid.n(), st, b.ops(), b.lzs(), b.res(), F.rmid.ptr(),
                       RowMidArgs{1 - s, OUT_VEC, 1.0, 1, 0, 0, 0, 0});
    }
    if (s == 1) launch_sign_fix(F.sg.n(), st, b.ops(), b.res(), F.sg.ptr(), 1);
    HIPCHK(hipGetLastError());
    // the singular values are read back when first asked for
    for (int i = 0; i < (int)b.ds.size(); ++i) {
        if (who && std::find(who->begin(), who->end(), i) == who->end()) continue;
        auto* d = b.ds[i];
        d->decomposed = true;
        d->sigma_ready = false;
        d->last_st = st;
    }
    return SSA_OK;
}

int fetch_kmask(ssa_decomp* d);

// U and sigma of the r leading eigenpairs of a block-Jacobi-rotated S: the
// eigenvalues (column norms) are ordered on the host, descending, ties by
// column.
int eig_take_big(Batch& b, ssa_decomp* d, int r) {
    std::vector<int> perm(d->L);
    for (int j = 0; j < (int)d->L; ++j) perm[j] = j;
    std::stable_sort(perm.begin(), perm.end(),
                     [&](int a, int c) { return d->eig_lam_h[a] > d->eig_lam_h[c]; });
    perm.resize(r);
    DevVec dperm;
    int rc;
    if ((rc = dperm.put(perm, b.st))) return rc;
    launch_bj_take(b.st, d->Sbig, (int)d->L, dperm.as<int>(), d->eig_lam, d->U, d->sigma, r);
    HIPCHK(hipGetLastError());
    return SSA_OK;
}

// Eigenpairs of S (resident in d->Sbig, L x L) by block one-sided Jacobi:
// sweeps of rounds that rotate disjoint pairs of column blocks until a
// whole sweep finds every pair orthogonal to 1e-13 relative to the column
// norms or below 1e-26 of the largest squared norm (at most 40 sweeps;
// beyond that the handle is returned with SSA_ENOCONV).  Then the column
// norms (the eigenvalues) and U, sigma of the r leading eigenpairs.
int eig_block_jacobi(Batch& b, ssa_decomp* d) {
    hipStream_t st = b.st;
    const int L = (int)d->L;
    const int nblk = (L + kBjW - 1) / kBjW, nb2 = nblk + (nblk & 1), P = nb2 / 2, rounds = nb2 - 1;
    // circle method over nb2 positions (the last one fixed); an odd block
    // count pairs one block with the empty block (-1) in each round
    std::vector<int2> pairs((size_t)rounds * P);
    for (int r = 0; r < rounds; ++r)
        for (int k = 0; k < P; ++k) {
            const int a = k == 0 ? nb2 - 1 : (r + k) % (nb2 - 1);
            const int c = k == 0 ? r : (r - k + nb2 - 1) % (nb2 - 1);
            pairs[(size_t)r * P + k] = make_int2(a < nblk ? a : -1, c < nblk ? c : -1);
        }
    DevVec dp, dJ, dflag;
    int rc;
    if ((rc = dp.put(pairs, st)) || (rc = dJ.reserve((size_t)P * kBjN * kBjN * sizeof(double))) ||
        (rc = dflag.reserve(2 * sizeof(int))))
        return rc;
    // scale: the largest squared column norm of S (>= lambda_1^2); Gram
    // entries below 1e-26 of it are not rotated away (they only couple
    // columns far below the eigenvalues that matter)
    launch_bj_norms(st, d->Sbig, L, d->eig_lam);
    d->eig_lam_h.assign(L, 0.0);
    HIPCHK(hipMemcpyAsync(d->eig_lam_h.data(), d->eig_lam, (size_t)L * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double nmax = 0.0;
    for (double v : d->eig_lam_h) nmax = std::max(nmax, v);
    const double floor_abs = 1e-26 * nmax * nmax;
    void* hb = nullptr;
    if ((rc = b.ctx->readback_buf(st, 2 * sizeof(int), &hb))) return rc;
    int sweeps = 0;
    bool conv = false;
    while (sweeps < 40 && !conv) {
        launch_fill_i32(st, dflag.as<int>(), 2, 0);
        for (int r = 0; r < rounds; ++r)
            launch_bj_round(st, d->Sbig, L, dp.as<int2>() + (size_t)r * P, P, dJ.as<double>(), dflag.as<int>(),
                            1e-13, floor_abs);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(hb, dflag.p, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        ++sweeps;
        conv = static_cast<int*>(hb)[0] == 0;
    }
    launch_bj_norms(st, d->Sbig, L, d->eig_lam);
    d->eig_lam_h.assign(L, 0.0);
    HIPCHK(hipMemcpyAsync(d->eig_lam_h.data(), d->eig_lam, (size_t)L * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    d->st.svd_sweeps = sweeps;
    d->st.converged = conv;
    if (!conv) d->status = fail(SSA_ENOCONV, "eigen method: block Jacobi reached its sweep limit");
    return eig_take_big(b, d, d->r);
}

// The eigen method (the paper's alternative for small windows): S = X X^T
// on the matrix cores straight from the cleaned grid, its eigenpairs by the
// one-sided Jacobi SVD of the projected-matrix kernel (S is symmetric
// positive semi-definite, so its left singular vectors are eigenvectors and
// its singular values the eigenvalues), U and sigma = sqrt(lambda) of the r
// leading ones.  The other side's vectors come from the finish pass.
int run_eigen(Batch& b, FinishLists& F) {
    hipStream_t st = b.st;
    int rc;
    ItemList I;
    for (size_t q = 0; q < b.ds.size(); ++q) {
        auto* d = b.ds[q];
        if ((rc = fetch_kmask(d))) return rc;
        std::vector<int> offL, offK;
        offL.reserve(d->L);
        offK.reserve(d->K);
        for (int a = 0; a < d->LA; ++a)
            for (int c = 0; c < d->LB; ++c)
                if (d->lmask_h[(size_t)a * d->LB + c]) offL.push_back(a * d->B + c);
        for (int a = 0; a < d->KA; ++a)
            for (int c = 0; c < d->KB; ++c)
                if (d->kmask_h[(size_t)a * d->KB + c]) offK.push_back(a * d->B + c);
        if ((long)offL.size() != d->L || (long)offK.size() != d->K || d->L > kEigMaxL)
            return fail(SSA_EINVAL, "eigen method: inconsistent cell sets");
        const int L = (int)d->L;
        const bool big = L > kMaxBasis;
        if (big && ((rc = d->dalloc(&d->Sbig, (long)L * L)) || (rc = d->dalloc(&d->eig_lam, L)))) return rc;
        const int nb = (L + 15) / 16, ntile = nb * (nb + 1) / 2;
        // about 2048 workgroups, each chunk at least 128 origins
        const int nchunk = (int)std::max<long>(1, std::min<long>(2048 / ntile + 1, (d->K + 127) / 128));
        DevVec dl, dk, part, out;
        if ((rc = dl.put(offL, st)) || (rc = dk.put(offK, st)) ||
            (rc = part.reserve((size_t)ntile * 256 * nchunk * sizeof(double))) ||
            (rc = out.reserve((size_t)ntile * 256 * sizeof(double))))
            return rc;
        {
            // flops of the Gram (upper-triangle tiles, 2 per multiply-add)
            ProfSpan p(b.ctx, "xgram", st, [&] { return 2.0 * ntile * 256.0 * (double)d->K; });
            launch_xgram(st, d->xc, dl.as<int>(), L, dk.as<int>(), d->K, nchunk, part.as<double>(),
                         out.as<double>(), big ? d->Sbig : d->Bm, big ? L : kMaxBasis);
        }
        HIPCHK(hipGetLastError());
        d->st.steps = 0;
        d->st.restarts = 0;
        d->st.basis = 0;
        d->st.converged = 1;
        d->st.max_resid = 0.0;
        // the DevVecs go back to the call's table cache, reused after the stream drains
        if (big) {
            if ((rc = eig_block_jacobi(b, d))) return rc;
        } else {
            I.h.push_back(Item{(int)q, 0, 0, 0});
        }
    }
    if (!I.h.empty()) {
        if ((rc = upload_lists({&I}, st))) return rc;
        const int L = (int)b.ds[I.h[0].inst]->L;
        launch_lz_svd(I.n(), st, b.lzs(), I.ptr(), L, 100);
        int rmax = 0;
        for (const Item& it : I.h) rmax = std::max(rmax, b.ds[it.inst]->r);
        launch_eig_take(I.n(), st, b.lzs(), b.res(), I.ptr(), L, rmax);
        HIPCHK(hipGetLastError());
    }
    return F.ready ? SSA_OK : finish_lists(b, F);
}

int seal_handle(ssa_decomp* d);

// Reconstruction of the same groups for every instance of the batch into
// internal-orientation device buffers recon[i] (ngroups x A x B).
int run_reconstruct(Batch& b, const std::vector<int>& gptr, const std::vector<int>& gidx,
                    const std::vector<double*>& recon) {
    hipStream_t st = b.st;
    const int ni = (int)b.ds.size();
    const int ng = (int)gptr.size() - 1;
    int rc;
    DevVec dgp, dgi;
    if ((rc = dgp.put(gptr, st)) || (rc = dgi.put(gidx, st))) return rc;
    // the group tables and output buffers are this call's: on every way out
    // the handles drop them (the uploaded descriptors keep them for the
    // queued kernels)
    struct Drop {
        Batch& b;
        ~Drop() {
            for (auto* d : b.ds) {
                d->rs.recon = nullptr;
                d->rs.gptr = nullptr;
                d->rs.gidx = nullptr;
            }
        }
    } drop{b};
    for (int i = 0; i < ni; ++i) {
        b.ds[i]->rs.recon = recon[i];
        b.ds[i]->rs.gptr = dgp.as<int>();
        b.ds[i]->rs.gidx = dgi.as<int>();
    }
    if ((rc = b.upload_descs())) return rc;
    std::vector<int> comps(gidx);
    std::sort(comps.begin(), comps.end());
    comps.erase(std::unique(comps.begin(), comps.end()), comps.end());
    const int nc = (int)comps.size();
    std::vector<int> all(ni);
    for (int i = 0; i < ni; ++i) all[i] = i;
    const auto* d0 = b.ds[0];
    ItemList a1, a2, c1, c2, out;
    if (d0->rowfam) {
        rows_items(a1, all, [&](int) { return 1; }, nc, &comps, row_group(b.cls, false));
        rows_items(out, all, [&](int i) { return b.ds[i]->A; }, ng);
        slot_pad(b, a1);
        slot_pad(b, out);
        if ((rc = a1.upload(st)) || (rc = out.upload(st))) return rc;
        launch_row_in(b.f64, b.cls, a1.n(), st, b.ops(), b.lzs(), b.res(), a1.ptr(),
                      RowInArgs{IN_VEC, 0, 0, DEST_T1, 1.0, 0});
        launch_copy_uspec(b.f64, a1.n(), st, b.ops(), a1.ptr());
        launch_rowfam_recon(b.f64, b.cls, out.n(), st, b.ops(), b.res(), out.ptr(), -1.0);   // spec_scale
    } else {
        rows_items(a1, all, [&](int i) { return b.ds[i]->LA; }, nc, &comps, row_group(b.cls, false));
        rows_items(a2, all, [&](int i) { return b.ds[i]->KA; }, nc, &comps, row_group(b.cls, false));
        rows_items(out, all, [&](int i) { return b.ds[i]->A; }, ng);
        for (int c : comps)
            for (int i : all)
                for (int t = 0; t < (b.ds[i]->P + b.TC - 1) / b.TC; ++t) c1.h.push_back(Item{i, t, c, 0});
        for (int g = 0; g < ng; ++g)
            for (int i : all)
                for (int t = 0; t < (b.ds[i]->P + b.TC - 1) / b.TC; ++t) c2.h.push_back(Item{i, t, g, 0});
        slot_pad(b, a1);
        slot_pad(b, a2);
        slot_pad(b, out);
        if ((rc = a1.upload(st)) || (rc = a2.upload(st)) || (rc = c1.upload(st)) || (rc = c2.upload(st)) ||
            (rc = out.upload(st)))
            return rc;
        launch_row_in(b.f64, b.cls, a1.n(), st, b.ops(), b.lzs(), b.res(), a1.ptr(),
                      RowInArgs{IN_VEC, 0, 0, DEST_T1, 1.0, 0});
        launch_col(b.f64, c1.n(), st, b.ops(), b.res(), c1.ptr(), ColArgs{COL_STORE, ROWS_S0, 0}, d0->MA, b.colcfg());
        launch_row_in(b.f64, b.cls, a2.n(), st, b.ops(), b.lzs(), b.res(), a2.ptr(),
                      RowInArgs{IN_VEC, 1, 0, DEST_T1, 1.0, 1});
        launch_col(b.f64, c2.n(), st, b.ops(), b.res(), c2.ptr(), ColArgs{COL_ACCUM, ROWS_S1, ROWS_ALL}, d0->MA,
                   b.colcfg());
        launch_row_out(b.f64, b.cls, out.n(), st, b.ops(), b.lzs(), b.res(), out.ptr(),
                       RowOutArgs{OUT_IMAGE, 0, -1.0, 0, 0, 0});   // each instance's spec_scale
    }
    HIPCHK(hipGetLastError());
    for (auto* d : b.ds) {
        d->last_st = st;
        (void)seal_handle(d);
    }
    return SSA_OK;
}

// Kernel class of a request.  Requests of one class advance together
// through the same kernels whatever their sizes and shapes (the descriptors
// carry each instance's geometry): operator family, precision, short side,
// row transform variant (row_word), column transform variant, and the basis
// and restart sizes of the bidiagonalisation.  The origin count can only
// shrink the basis of small problems; run_planned splits a batch again on
// the sizes that hold after the count.
using GeoKey = std::tuple<int, int, int, int, int, int, int>;
int col_key(int MA) {
    if (MA <= 1) return 0;                            // row family: no column pass
    if (col_fast_logn(MA)) return MA;                 // register kernel of that length
    return (MA & (MA - 1)) == 0 ? -2 : -1;            // LDS kernel, radix-2 or mixed plan
}
GeoKey geo_key(const ssa_decomp* d) {
    const int side = plan_side(d);
    const long nshort = side == 0 ? d->L : (long)d->KA * d->KB;   // the origin box bounds |K|
    const int m = basis_size(nshort, d->r);
    return GeoKey{(int)d->rowfam, d->f64 ? 0 : d->q32 ? 2 : 1, side, row_word(d->nh, d->f64), col_key(d->MA), m,
                  restart_keep(m, d->r)};
}

int ensure_sub_streams(ssa_ctx* ctx, int n) {
    std::lock_guard<std::mutex> g(ctx->mu);
    while ((int)ctx->sub_st.size() < n) {
        hipStream_t s = nullptr;
        HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        ctx->sub_st.push_back(s);
    }
    return SSA_OK;
}

// Decompose planned and uploaded instances of one geometry group on stream
// st (setup, spectrum, bidiagonalisation, other-side vectors).  st[i]
// receives each instance's status.
void run_planned(ssa_ctx* ctx, const std::vector<ssa_decomp*>& grp, hipStream_t stream, std::vector<int>& st) {
    const int n = (int)grp.size();
    st.assign(n, SSA_OK);
    if (n == 0) return;
    for (auto* d : grp) d->last_st = stream;
    Batch b(ctx, stream);
    b.ds = grp;
    b.f64 = b.ds[0]->f64;
    b.rowfam = b.ds[0]->rowfam;
    b.cls = row_word(b.ds[0]->nh, b.f64);
    b.set_col(ctx->tile_for(b.f64, b.ds[0]->MA));
    auto t0 = Clock::now();
    int rc = run_setup(b);
    if (rc) {
        st.assign(n, rc);
        return;
    }
    // drop instances whose shapes failed
    std::vector<ssa_decomp*> ok;
    for (int i = 0; i < n; ++i) {
        if (grp[i]->status != SSA_OK) st[i] = grp[i]->status;
        else ok.push_back(grp[i]);
    }
    if (ok.empty()) return;
    // sub-batches of equal basis and restart size (the origin count fixes
    // the short side's size)
    std::map<std::pair<int, int>, std::vector<ssa_decomp*>> parts;
    for (auto* d : ok) {
        choose_side(d);
        if (d->eigen) {
            // S lives on the window side
            d->side = 0;
            d->nshort = d->L;
            d->nlong = d->K;
            parts[{0, 0}].push_back(d);
            continue;
        }
        const int m = basis_size(d->nshort, d->r);
        parts[{m, restart_keep(m, d->r)}].push_back(d);
    }
    double t_setup = ms_since(t0);
    for (auto& kv : parts) {
        b.ds = kv.second;
        auto t1 = Clock::now();
        rc = run_alloc_spectrum(b);
        if (!rc) (void)hipStreamSynchronize(stream);
        const double t_spec = ms_since(t1);
        auto t2 = Clock::now();
        FinishLists F;
        if (!rc) {
            const int slots = ctx->slots;
            if (b.ds[0]->eigen)
                rc = run_eigen(b, F);
            else if (slots > 0 && (int)b.ds.size() > slots)
                rc = run_lanczos_cont(b, step_limit(), slots, [&] { return finish_lists(b, F); });
            else
                rc = run_lanczos(b, step_limit(), [&] { return finish_lists(b, F); });
        }
        const double t_lz = ms_since(t2);
        auto t3 = Clock::now();
        if (!rc) rc = run_finish(b, F);
        const double t_fin = ms_since(t3);
        const double nb = (double)b.ds.size();
        for (auto* d : b.ds) {
            d->st.ms_setup = (t_setup + t_spec) / nb;
            d->st.ms_lanczos = t_lz / nb;
            d->st.ms_finish = t_fin / nb;
            d->st.side = d->side;
            d->st.batch = (int)b.ds.size();
            if (rc) d->status = rc;
        }
    }
    for (int i = 0; i < n; ++i)
        if (grp[i]->status != SSA_OK && st[i] == SSA_OK) st[i] = grp[i]->status;
}

int decompose_core(ssa_ctx* ctx, int n, const ssa_request* reqs, ssa_decomp** out, int* status, bool dev,
                   int nh_force, int ma_force);
int wait_handle(ssa_decomp* d);
std::mutex g_len_tune_mu;   // one length tuning at a time (it decomposes, so it cannot hold tune_mu)

// Length tuner: the first request of a (precision, natural transform
// length) class with a power-of-two alternative (row half-lengths up to
// 512, column lengths up to 1024, at most 30% more points) is decomposed at
// both lengths, twice each; the length of the faster second run is kept for
// the process (every context pads that class alike) and appended to the
// context's tune cache.  Any length M >= N gives the same products and
// averages up to rounding.  Off unless the context was created with
// SHSSA_LEN_TUNE set: a power-of-two length has a register kernel of its own,
// so requests of different natural lengths that share one LDS kernel class
// (and one batch) would be split into several classes; the tuner suits
// workloads of uniform sizes.
int tune_lengths(ssa_ctx* ctx, int n, const ssa_request* reqs, bool dev) {
    if (!ctx->len_tune) return SSA_OK;
    std::lock_guard<std::mutex> tune_lock(g_len_tune_mu);
    for (int i = 0; i < n; ++i) {
        ssa_decomp probe;
        if (plan_request(ctx, reqs[i], &probe) != SSA_OK) continue;
        for (int kind = 0; kind < 2; ++kind) {
            if (kind == 1 && probe.rowfam) continue;
            const int n0 = kind == 0 ? probe.nh0 : probe.MA0;
            const int alt = len_alternative(kind, n0, kind == 0 ? (probe.B + 1) / 2 : probe.A);
            if (!alt || len_choice(kind, probe.f64, n0).second) continue;
            double best = 1e30;
            int choice = n0;
            for (int cand : {n0, alt}) {
                double t = 0.0;
                for (int rep = 0; rep < 2; ++rep) {
                    ssa_decomp* h = nullptr;
                    int stt = SSA_OK;
                    const auto t0 = Clock::now();
                    int rc = decompose_core(ctx, 1, &reqs[i], &h, &stt, dev, kind == 0 ? cand : 0,
                                            kind == 1 ? cand : 0);
                    if (!rc && h) rc = wait_handle(h);
                    t = ms_since(t0);
                    delete h;
                    if (rc || stt) return SSA_OK;   // leave the class untuned; the request reports its own error
                }
                if (std::getenv("SHSSA_TUNE_LOG"))
                    std::fprintf(stderr, "length tuner: %s f64 %d natural %d -> %d: %.3f ms\n", kind ? "col" : "row",
                                 (int)probe.f64, n0, cand, t);
                if (t < best) { best = t; choice = cand; }
            }
            {
                std::lock_guard<std::mutex> g(g_len_mu);
                g_len_tc[std::make_tuple(kind, (int)probe.f64, n0)] = choice;
            }
            {
                std::lock_guard<std::mutex> g(ctx->tune_mu);
                ctx->tune_save(kind ? "collen" : "rowlen", (int)probe.f64, n0, choice);
            }
        }
    }
    return SSA_OK;
}

int decompose_many(ssa_ctx* ctx, int n, const ssa_request* reqs, ssa_decomp** out, int* status, bool dev) {
    if (!ctx || n < 0 || (n > 0 && (!reqs || !out))) return fail(SSA_EINVAL, "bad arguments");
    (void)tune_lengths(ctx, n, reqs, dev);
    return decompose_core(ctx, n, reqs, out, status, dev, 0, 0);
}

int decompose_core(ssa_ctx* ctx, int n, const ssa_request* reqs, ssa_decomp** out, int* status, bool dev,
                   int nh_force, int ma_force) {
    if (!ctx || n < 0 || (n > 0 && (!reqs || !out))) return fail(SSA_EINVAL, "bad arguments");
    g_tables_ctx = ctx;
    TableScope tables(ctx, ctx->st);
    std::vector<std::unique_ptr<ssa_decomp>> ds(n);
    std::vector<int> st(n, SSA_OK);
    std::map<GeoKey, std::vector<int>> groups;
    std::vector<CopyJob> jobs;
    for (int i = 0; i < n; ++i) {
        out[i] = nullptr;
        ds[i].reset(new ssa_decomp());
        st[i] = plan_request(ctx, reqs[i], ds[i].get(), nh_force, ma_force);
        if (st[i] == SSA_OK) st[i] = upload_request(reqs[i], ds[i].get(), dev, ctx->st, &jobs);
        if (st[i] == SSA_OK) groups[geo_key(ds[i].get())].push_back(i);
    }
    // the device inputs' copies, all in one launch (before the set-up reads them)
    DevVec jd;
    if (!jobs.empty()) {
        long mx = 0;
        for (const CopyJob& j : jobs) mx = std::max(mx, j.bytes);
        if (jobs.size() <= 65535 && jd.put(jobs, ctx->st) == SSA_OK) {
            launch_copy_jobs(ctx->st, jd.as<CopyJob>(), (int)jobs.size(), mx);
        } else {
            for (const CopyJob& j : jobs)
                HIPCHK(hipMemcpyAsync(j.dst, j.src, j.bytes, hipMemcpyDeviceToDevice, ctx->st));
        }
    }
    // Concurrent sub-batches (SHSSA_BATCH_STREAMS = 2..4) gain about 5% on
    // the 512^2 batch-64 workload but share the GPU between product kernels
    // of different sub-batches; one stream is the default.
    int nsub = 1;
    if (const char* e = std::getenv("SHSSA_BATCH_STREAMS")) nsub = std::max(1, std::min(4, std::atoi(e)));
    for (auto& kv : groups) {
        std::vector<ssa_decomp*> grp;
        for (int i : kv.second) grp.push_back(ds[i].get());
        std::vector<int> gst;
        const int ns = (int)grp.size() >= 16 ? nsub : 1;
        if (ns == 1) {
            run_planned(ctx, grp, ctx->st, gst);
        } else {
            // Concurrent sub-batches on their own streams: one sub-batch's
            // latency-bound phases (small SVDs, converged-instance tails,
            // launch gaps) overlap another's products.
            int rc = SSA_OK;
            if ((rc = ensure_sub_streams(ctx, ns))) {
                for (int i : kv.second) st[i] = rc;
                continue;
            }
            HIPCHK(hipStreamSynchronize(ctx->st));   // inputs uploaded on the context stream
            std::vector<std::vector<ssa_decomp*>> parts(ns);
            for (size_t k = 0; k < grp.size(); ++k) parts[k * ns / grp.size()].push_back(grp[k]);
            std::vector<std::vector<int>> pst(ns);
            std::vector<std::thread> th;
            for (int q = 1; q < ns; ++q)
                th.emplace_back([&, q] {
                    (void)hipSetDevice(ctx->device);
                    g_tables_ctx = ctx;
                    TableScope tables(ctx, ctx->sub_st[q]);
                    run_planned(ctx, parts[q], ctx->sub_st[q], pst[q]);
                });
            {
                std::vector<std::pair<void*, size_t>> cache;
                auto* prev = g_table_cache;
                g_table_cache = &cache;
                run_planned(ctx, parts[0], ctx->sub_st[0], pst[0]);
                {
                    std::lock_guard<std::mutex> g(ctx->mu);
                    ctx->defer(cache, ctx->sub_st[0]);
                }
                g_table_cache = prev;
            }
            for (auto& t : th) t.join();
            // the handles leave the sub-batch streams complete
            for (int q = 0; q < ns; ++q) HIPCHK(hipStreamSynchronize(ctx->sub_st[q]));
            for (auto* d : grp) d->last_st = nullptr;
            for (int q = 0; q < ns; ++q) gst.insert(gst.end(), pst[q].begin(), pst[q].end());
        }
        for (size_t k = 0; k < kv.second.size(); ++k) st[kv.second[k]] = gst[k];
    }
    for (int i = 0; i < n; ++i) {
        if (status) status[i] = st[i];
        if (st[i] == SSA_OK || st[i] == SSA_ENOCONV) {
            (void)seal_handle(ds[i].get());
            out[i] = ds[i].release();
        }
    }
    return SSA_OK;
}

// Wait for the work queued on a handle (library calls return before it
// completes); its device results are then final.
int wait_handle(ssa_decomp* d) {
    if (d->last_st) HIPCHK(hipStreamSynchronize(d->last_st));
    if (d->last_ev) HIPCHK(hipEventSynchronize(d->last_ev));
    return SSA_OK;
}

// End of a library call that queued work on d: replace the stream by an
// event recorded behind the work (the caller may destroy or replace the
// stream afterwards).
int seal_handle(ssa_decomp* d) {
    if (!d->last_st) return SSA_OK;
    if (!d->last_ev) {
        std::lock_guard<std::mutex> g(d->ctx->mu);
        d->last_ev = d->ctx->take_event();
    }
    if (!d->last_ev || hipEventRecord(d->last_ev, d->last_st) != hipSuccess) {
        HIPCHK(hipStreamSynchronize(d->last_st));   // no event: wait instead
    }
    d->last_st = nullptr;
    return SSA_OK;
}

// Convert internal compact vectors to the caller's boxes (NaN off the set).
int fetch_kmask(ssa_decomp* d) {
    if (!d->kmask_h.empty()) return SSA_OK;
    d->kmask_h.resize((size_t)d->KA * d->KB);
    HIPCHK(hipMemcpy(d->kmask_h.data(), d->kmask, d->kmask_h.size(), hipMemcpyDeviceToHost));
    return SSA_OK;
}

// For a set box (internal BA x BB) and its mask, call fn(compact index,
// caller row, caller col) for every cell in internal row-major order.
template <typename F>
void walk_set(const ssa_decomp* d, int BA, int BB, const uint8_t* mask, F fn) {
    long idx = 0;
    for (int a = 0; a < BA; ++a)
        for (int b = 0; b < BB; ++b) {
            if (mask && !mask[(size_t)a * BB + b]) continue;
            const int i = d->tr ? b : a, j = d->tr ? a : b;
            fn(idx++, i, j);
        }
}

}  // namespace

// ---------------------------------------------------------------------------
// serving: asynchronous requests, admission, batching over several streams
// ---------------------------------------------------------------------------

// One submitted request.  The inputs are copied at submission; the handle
// is planned (host-only) at once so that admission and batching know its
// geometry and size.
struct ServeReq {
    uint64_t ticket = 0;
    std::vector<double> x;
    std::vector<uint8_t> mask, wmask;
    ssa_request q{};
    std::vector<int> gp, gi;
    std::unique_ptr<ssa_decomp> d;
    size_t est = 0;
    GeoKey key;
    double t_submit = 0.0, t_start = 0.0, t_done = 0.0;   // ms since the server started
    int status = SSA_EBUSY;   // written by the worker while it runs the request
    bool done = false;        // set under the server lock once the request has finished
    std::vector<double> recon;   // ngroups x nx x ny (caller layout) once done
};

struct CoopState;

struct Server {
    std::shared_ptr<CoopState> coop;   // cooperative mode: no threads, the callers' waits drive the work
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::shared_ptr<ServeReq>> pending;
    std::map<uint64_t, std::shared_ptr<ServeReq>> reqs;   // until taken
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    Clock::time_point t0 = Clock::now();
    uint64_t next = 1;
    size_t reserved = 0;      // admitted estimates not yet released
    int running = 0;          // batches in flight (cooperative mode: admitted requests)
    int max_batch = 64;
    bool stop = false;
    double now() const { return ms_since(t0); }
};

// Device bytes one request will hold while it runs (an upper bound: the
// origin box stands in for the origin set, plus size-class slack).
size_t estimate_bytes(const ssa_decomp* d, int ngroups) {
    const double n = (double)d->A * d->B, ce = d->f64 ? 16.0 : 8.0;
    const double kbox = (double)d->KA * d->KB, L = (double)d->L;
    const double nshort = std::min(L, kbox), nlong = std::max(L, kbox);
    const double nslot = std::max(1, d->r);
    const double xh = d->rowfam ? (double)d->A * d->ldp : (double)d->ldp * d->MA;
    const double us = d->rowfam ? (double)d->P : (double)d->P * d->MA;
    double b = 27.0 * n + 5.0 * kbox + 5.0 * d->LA * d->LB;           // x, masks, xc, W, prefix sums
    b += xh * ce + 2.0 * d->A * d->ldp * ce * nslot + us * ce * nslot;  // spectrum, row/column slots
    b += 2.0 * nlong * (d->f64 ? 8.0 : 4.0);                            // long vectors
    b += nshort * (2.0 * kMaxBasis + 4.0) * 8.0;                        // basis, rotation scratch, w
    if (d->q32) b += nshort * (kMaxBasis + 1.0) * 4.0;                  // FP32 copy of the basis
    b += (L + kbox) * d->r * 8.0;                                       // U, V
    b += (double)ngroups * n * 8.0;                                     // reconstruction
    return (size_t)(1.3 * b) + (4u << 20);
}

void fill_batch(Batch& b, ssa_ctx* ctx, const std::vector<ssa_decomp*>& ds) {
    b.ds = ds;
    b.f64 = ds[0]->f64;
    b.rowfam = ds[0]->rowfam;
    b.cls = row_word(ds[0]->nh, b.f64);
    b.set_col(ctx->tile_for(b.f64, ds[0]->MA));
}

// Decompose and reconstruct one batch of requests of equal geometry on
// stream st; results land in the requests.
void serve_batch(ssa_ctx* ctx, std::vector<std::shared_ptr<ServeReq>>& batch, hipStream_t st) {
    std::vector<ssa_decomp*> grp;
    std::vector<ServeReq*> live;
    for (auto& r : batch) {
        r->status = upload_request(r->q, r->d.get(), false, st);
        if (r->status == SSA_OK) {
            grp.push_back(r->d.get());
            live.push_back(r.get());
        }
    }
    std::vector<int> gst;
    run_planned(ctx, grp, st, gst);
    // reconstructions, one launch sequence per distinct group list
    std::vector<ServeReq*> ok;
    for (size_t k = 0; k < live.size(); ++k) {
        live[k]->status = gst[k];
        if (gst[k] == SSA_OK && live[k]->gp.size() > 1) ok.push_back(live[k]);
    }
    std::vector<char> done(ok.size(), 0);
    for (size_t a = 0; a < ok.size(); ++a) {
        if (done[a]) continue;
        std::vector<ServeReq*> same;
        for (size_t c = a; c < ok.size(); ++c)
            if (!done[c] && ok[c]->gp == ok[a]->gp && ok[c]->gi == ok[a]->gi) {
                same.push_back(ok[c]);
                done[c] = 1;
            }
        const int ng = (int)same[0]->gp.size() - 1;
        std::vector<ssa_decomp*> ds;
        std::vector<double*> bufs;
        int rc = SSA_OK;
        for (auto* r : same) {
            double* buf = nullptr;
            if ((rc = r->d->dalloc(&buf, (long)ng * r->d->A * r->d->B))) break;
            ds.push_back(r->d.get());
            bufs.push_back(buf);
        }
        if (!rc) {
            Batch b(ctx, st);
            fill_batch(b, ctx, ds);
            rc = run_reconstruct(b, same[0]->gp, same[0]->gi, bufs);
        }
        for (size_t k = 0; k < same.size(); ++k) {
            ServeReq* r = same[k];
            if (rc || k >= bufs.size()) {
                r->status = rc ? rc : SSA_ENOMEM;
                continue;
            }
            const ssa_decomp* d = r->d.get();
            const long n = (long)d->A * d->B;
            std::vector<double> t((size_t)n * ng);
            if (hipMemcpyAsync(t.data(), bufs[k], t.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                r->status = fail(SSA_EDEVICE, "reconstruction copy");
                continue;
            }
            r->recon.resize(t.size());
            if (!d->tr) {
                r->recon.swap(t);
            } else {
                for (int g = 0; g < ng; ++g)
                    for (int a2 = 0; a2 < d->A; ++a2)
                        for (int b2 = 0; b2 < d->B; ++b2)
                            r->recon[g * n + (long)b2 * d->A + a2] = t[g * n + (long)a2 * d->B + b2];
            }
        }
    }
    (void)hipStreamSynchronize(st);
    // handed to the caller complete: nothing refers to the worker's stream
    for (auto& r : batch)
        if (r->d) r->d->last_st = nullptr;
}

// Admission: the oldest request starts when its estimate fits the budget
// beside the running batches (a request that cannot fit even alone is
// refused at submission); compatible waiting requests join its batch.
bool serve_can_start(const Server& s, size_t budget) {
    if (s.pending.empty()) return false;
    return budget == 0 || s.running == 0 || s.reserved + s.pending.front()->est <= budget;
}

void serve_worker(ssa_ctx* ctx, int w) {
    Server& S = *ctx->srv;
    (void)hipSetDevice(ctx->device);
    g_tables_ctx = ctx;
    std::vector<std::pair<void*, size_t>> cache;
    g_table_cache = &cache;
    const hipStream_t st = S.streams[w];
    for (;;) {
        std::vector<std::shared_ptr<ServeReq>> batch;
        size_t est = 0;
        {
            std::unique_lock<std::mutex> lk(S.mu);
            S.cv.wait(lk, [&] { return S.stop || serve_can_start(S, ctx->budget); });
            if (S.stop) break;
            auto r0 = S.pending.front();
            S.pending.pop_front();
            batch.push_back(r0);
            est = r0->est;
            for (auto it = S.pending.begin(); it != S.pending.end() && (int)batch.size() < S.max_batch;) {
                if ((*it)->key == r0->key && (ctx->budget == 0 || S.reserved + est + (*it)->est <= ctx->budget)) {
                    est += (*it)->est;
                    batch.push_back(*it);
                    it = S.pending.erase(it);
                } else {
                    ++it;
                }
            }
            S.reserved += est;
            S.running++;
            const double t = S.now();
            for (auto& r : batch) r->t_start = t;
        }
        serve_batch(ctx, batch, st);
        flush_table_cache(ctx);
        {
            std::lock_guard<std::mutex> lk(S.mu);
            S.reserved -= est;
            S.running--;
            const double t = S.now();
            for (auto& r : batch) {
                r->t_done = t;
                if (r->status == SSA_EBUSY) r->status = SSA_EDEVICE;
                r->done = true;
            }
        }
        S.cv.notify_all();
    }
    flush_table_cache(ctx);
    g_table_cache = nullptr;
}

// Starts the serving threads once per context; concurrent first calls of
// ssa_submit from several threads start one server.
// ---------------------------------------------------------------------------
// cooperative serving (the default): ssa_poll and ssa_wait drive the
// requests on the context's stream, in the calling thread, one restart
// cycle at a time
// ---------------------------------------------------------------------------

// The requests of one kernel class (geometry, basis and restart size) that
// advance together.  At each cycle boundary waiting requests take the slots
// of finished ones and begin from their start vectors, and finished ones
// leave the batch with their results: each instance keeps its own step
// counter [j, jstart] on the device, and the cycle plan of basis_size and
// restart_keep puts every instance's boundaries on common ones, so it runs
// the steps, restarts and reductions it would run alone.
struct CoopBatch {
    GeoKey key;
    int m = 0, kk = 0;
    Batch b;
    struct Inst {
        std::shared_ptr<ServeReq> r;
        int* ctr = nullptr;   // [j, jstart] (a block of the handle)
        int steps = 0, restarts = 0, jh = 0, cycles = 0, bdrest = 0;
        bool active = false;
    };
    std::vector<Inst> in;   // in[i] runs b.ds[i]
    bool dirty = true;      // descriptors changed since the last upload
    StepLists lists;        // item lists of the active set lists_for (kept while it stays)
    std::vector<int> lists_for;
    explicit CoopBatch(ssa_ctx* ctx) : b(ctx) {}
};

struct CoopState {
    std::vector<std::unique_ptr<CoopBatch>> batches;
};

// A request leaves the server with its status (results in place when OK).
void coop_done(Server& S, const std::shared_ptr<ServeReq>& r, int status) {
    std::lock_guard<std::mutex> lk(S.mu);
    r->status = status;
    r->t_done = S.now();
    r->done = true;
    S.reserved -= r->est;
    S.running--;
}

// The reconstructions of a finished request (its groups, caller layout).
int coop_reconstruct(ssa_ctx* ctx, ServeReq* r) {
    if (r->gp.size() < 2) return SSA_OK;
    ssa_decomp* d = r->d.get();
    const int ng = (int)r->gp.size() - 1;
    const long n = (long)d->A * d->B;
    double* buf = nullptr;
    int rc;
    if ((rc = d->dalloc(&buf, (long)ng * n))) return rc;
    {
        Batch b(ctx, ctx->st);
        fill_batch(b, ctx, {d});
        if ((rc = run_reconstruct(b, r->gp, r->gi, {buf}))) return rc;
    }
    std::vector<double> t((size_t)n * ng);
    HIPCHK(hipMemcpyAsync(t.data(), buf, t.size() * 8, hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
    r->recon.resize(t.size());
    if (!d->tr) {
        r->recon.swap(t);
    } else {
        for (int g = 0; g < ng; ++g)
            for (int a = 0; a < d->A; ++a)
                for (int c = 0; c < d->B; ++c) r->recon[g * n + (long)c * d->A + a] = t[g * n + (long)a * d->B + c];
    }
    return SSA_OK;
}

// Admission: waiting requests in arrival order while their estimates fit
// the budget beside the admitted ones (the first one always, when nothing
// runs), set up on the context's stream and added to their class's batch.
int coop_admit(ssa_ctx* ctx, Server& S, CoopState& C) {
    std::vector<std::shared_ptr<ServeReq>> take;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        while (!S.pending.empty()) {
            auto r = S.pending.front();
            if (ctx->budget && S.running > 0 && S.reserved + r->est > ctx->budget) break;
            S.pending.pop_front();
            S.reserved += r->est;
            S.running++;
            r->t_start = S.now();
            take.push_back(r);
        }
    }
    if (take.empty()) return SSA_OK;
    const hipStream_t st = ctx->st;
    std::map<GeoKey, std::vector<std::shared_ptr<ServeReq>>> groups;
    for (auto& r : take) {
        const int rc = upload_request(r->q, r->d.get(), false, st);
        if (rc) coop_done(S, r, rc);
        else groups[r->key].push_back(r);
    }
    for (auto& kv : groups) {
        std::vector<ssa_decomp*> ds;
        for (auto& r : kv.second) ds.push_back(r->d.get());
        int rc;
        {
            Batch t(ctx, st);
            fill_batch(t, ctx, ds);
            rc = run_setup(t);
        }
        std::map<std::pair<int, int>, std::vector<std::shared_ptr<ServeReq>>> parts;
        for (auto& r : kv.second) {
            ssa_decomp* d = r->d.get();
            if (rc || d->status != SSA_OK) {
                coop_done(S, r, rc ? rc : d->status);
                continue;
            }
            choose_side(d);
            const int m = basis_size(d->nshort, d->r);
            parts[{m, restart_keep(m, d->r)}].push_back(r);
        }
        for (auto& pv : parts) {
            std::vector<ssa_decomp*> pd;
            for (auto& r : pv.second) pd.push_back(r->d.get());
            std::vector<int*> ctrs(pd.size(), nullptr);
            int prc;
            {
                Batch t(ctx, st);
                fill_batch(t, ctx, pd);
                prc = run_alloc_spectrum(t);
                for (size_t k = 0; k < pd.size() && !prc; ++k) prc = pd[k]->dalloc(&ctrs[k], 2);
            }
            if (prc) {
                for (auto& r : pv.second) coop_done(S, r, prc);
                continue;
            }
            CoopBatch* B = nullptr;
            for (auto& cb : C.batches)
                if (cb->key == kv.first && cb->m == pv.first.first && cb->kk == pv.first.second) B = cb.get();
            if (!B) {
                C.batches.emplace_back(new CoopBatch(ctx));
                B = C.batches.back().get();
                B->key = kv.first;
                B->m = pv.first.first;
                B->kk = pv.first.second;
            }
            for (size_t k = 0; k < pd.size(); ++k) {
                pd[k]->last_st = st;
                pd[k]->lz.step = ctrs[k];
                pd[k]->st.basis = B->m;
                B->b.ds.push_back(pd[k]);
                CoopBatch::Inst I;
                I.r = pv.second[k];
                I.ctr = ctrs[k];
                B->in.push_back(I);
            }
            fill_batch(B->b, ctx, B->b.ds);
            B->dirty = true;
        }
    }
    return SSA_OK;
}

// One restart cycle of a batch: waiting instances take free slots, the
// active ones take m - kk steps (m on their first cycle, in q shorter
// cycles of the same length), and at the boundary the instances whose
// cycle ends are tested, restarted or finished.
int coop_cycle(ssa_ctx* ctx, Server& S, CoopBatch& B, int slots) {
    Batch& b = B.b;
    const hipStream_t st = b.st;
    const int m = B.m, kk = B.kk, c = m - kk;
    int rc;
    int nact = 0;
    for (auto& I : B.in) nact += I.active;
    std::vector<int> joiners;
    for (int i = 0; i < (int)B.in.size() && nact < slots; ++i)
        if (!B.in[i].active) {
            B.in[i].active = true;
            B.in[i].jh = 0;
            joiners.push_back(i);
            ++nact;
        }
    if (B.dirty) {
        if ((rc = b.upload_descs())) return rc;
        B.dirty = false;
        B.lists_for.clear();   // positions may have changed
    }
    if (!joiners.empty()) {
        ItemList Z, I;
        for (int i : joiners) {
            for (int k = 0; k < b.ds[i]->lz.nblk; ++k) Z.h.push_back(Item{i, k, 0, 0});
            I.h.push_back(Item{i, 0, 0, 0});
        }
        if ((rc = upload_lists({&Z, &I}, st))) return rc;
        launch_lz_start(Z.n(), st, b.lzs(), Z.ptr(), 0ULL);   // each instance's own seed
        launch_step_set(I.n(), st, b.lzs(), I.ptr(), 0, 0);
    }
    std::vector<int> act;
    for (int i = 0; i < (int)B.in.size(); ++i)
        if (B.in[i].active) act.push_back(i);
    if (act.empty()) return SSA_OK;
    StepLists& SL = B.lists;
    if (act != B.lists_for) {
        build_step_lists(b, act, SL);
        if ((rc = upload_step_lists(SL, st))) return rc;
        B.lists_for = act;
    }
    for (int k = 0; k < c; ++k) {
        launch_step(b, SL, kStepDev, kStepDev, IN_LZ_STEP);
        launch_step_next_inst(SL.inst.n(), st, b.lzs(), SL.inst.ptr());
    }
    HIPCHK(hipGetLastError());
    std::vector<int> ends;
    for (int i : act) {
        B.in[i].jh += c;
        if (B.in[i].jh == m) ends.push_back(i);
    }
    if (ends.empty()) return SSA_OK;
    const int ni = (int)b.ds.size();
    int rmax = 0;
    for (auto* d : b.ds) rmax = std::max(rmax, d->r);
    {
        ItemList N, I;
        for (int i : ends) {
            for (int k = 0; k < b.ds[i]->lz.nblk; ++k) N.h.push_back(Item{i, k, 0, 0});
            I.h.push_back(Item{i, 0, 0, 0});
        }
        if ((rc = upload_lists({&N, &I}, st))) return rc;
        launch_lz_normalize(N.n(), st, b.lzs(), N.ptr(), m);
        launch_lz_svd(I.n(), st, b.lzs(), I.ptr(), m, 40);
    }
    HIPCHK(hipGetLastError());
    const size_t fb = (size_t)ni * 4 * sizeof(int), bb = (size_t)ni * 2 * sizeof(double);
    if (!b.dflag.p || b.dflag.cap < fb + bb) {
        std::vector<char> z(fb + bb, 0);
        if ((rc = b.dflag.put(z, st))) return rc;
    }
    char* dv = b.dflag.as<char>();
    launch_gather_flags(ni, st, b.lzs(), reinterpret_cast<int*>(dv), reinterpret_cast<double*>(dv + fb));
    void* hb = nullptr;
    if ((rc = ctx->readback_buf(st, fb + bb, &hb))) return rc;
    HIPCHK(hipMemcpyAsync(hb, dv, fb + bb, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<int> flags(4 * (size_t)ni);
    std::vector<double> betas(2 * (size_t)ni);
    std::memcpy(flags.data(), hb, fb);
    std::memcpy(betas.data(), static_cast<char*>(hb) + fb, bb);
    const int max_steps = step_limit();
    std::vector<int> done, cont, fresh;
    for (int i : ends) {
        auto& I = B.in[i];
        I.steps += m - (I.cycles == 0 ? 0 : kk);
        ++I.cycles;
        auto* d = b.ds[i];
        d->st.svd_sweeps += flags[4 * i + 1];
        const bool ok = flags[4 * i] != 0;
        const bool bd = flags[4 * i + 2] != 0;
        if (bd && I.bdrest < 2 && I.steps < max_steps) {
            I.bdrest++;
            I.restarts++;
            fresh.push_back(i);
            cont.push_back(i);
            continue;
        }
        if (ok || bd || I.steps >= max_steps) {
            done.push_back(i);
            d->st.converged = ok || bd;
            d->st.steps = I.steps;
            d->st.restarts = I.restarts;
            d->st.max_resid = betas[2 * i + 1];
            d->st.side = d->side;
            d->st.batch = nact;
            if (!(ok || bd)) d->status = SSA_ENOCONV;
        } else {
            cont.push_back(i);
            I.restarts++;
        }
    }
    if (!cont.empty()) {
        // the random restart of a breakdown draws from the instance's own
        // cycle count
        std::map<int, std::vector<int>> by_cycle;
        for (int i : cont) {
            const bool f = std::find(fresh.begin(), fresh.end(), i) != fresh.end();
            by_cycle[f ? B.in[i].cycles : -1].push_back(i);
        }
        for (auto& kv : by_cycle) {
            const std::vector<int>& grp = kv.second;
            if ((rc = launch_restart(b, grp, kv.first < 0 ? std::vector<int>{} : grp, m, kk,
                                     kv.first < 0 ? 0 : kv.first)))
                return rc;
        }
        ItemList I2;
        for (int i : cont) {
            I2.h.push_back(Item{i, 0, 0, 0});
            B.in[i].jh = kk;
        }
        if ((rc = upload_lists({&I2}, st))) return rc;
        launch_step_set(I2.n(), st, b.lzs(), I2.ptr(), kk, kk);
    }
    if (done.empty()) return SSA_OK;
    if ((rc = lanczos_outputs(b, done, m, rmax))) return rc;
    {
        FinishLists F;
        if ((rc = run_finish(b, F, &done))) return rc;
    }
    HIPCHK(hipGetLastError());
    // results of the finished requests, then they leave the batch
    std::vector<std::pair<std::shared_ptr<ServeReq>, int>> fin;
    for (int i : done) {
        auto r = B.in[i].r;
        ssa_decomp* d = r->d.get();
        int status = d->status == SSA_ENOCONV ? SSA_ENOCONV : SSA_OK;
        if (const int e = coop_reconstruct(ctx, r.get())) status = e;
        if (hipStreamSynchronize(st) != hipSuccess) status = SSA_EDEVICE;
        else d->last_st = nullptr;   // complete: nothing queued refers to it
        fin.emplace_back(r, status);
    }
    std::vector<ssa_decomp*> keep_ds;
    std::vector<CoopBatch::Inst> keep;
    for (int i = 0; i < ni; ++i)
        if (std::find(done.begin(), done.end(), i) == done.end()) {
            keep_ds.push_back(b.ds[i]);
            keep.push_back(B.in[i]);
        }
    b.ds.swap(keep_ds);
    B.in.swap(keep);
    B.dirty = true;
    for (auto& f : fin) coop_done(S, f.first, f.second);
    return SSA_OK;
}

// One round of the cooperative server: admissions, then one cycle of the
// batch that holds the oldest request (requests are served in arrival
// order, each batch carrying the later requests of its class that have
// joined it).  Caller holds the context's call lock.
int coop_advance(ssa_ctx* ctx) {
    Server& S = *ctx->srv;
    CoopState& C = *S.coop;
    g_tables_ctx = ctx;
    TableScope tables(ctx, ctx->st);
    int rc;
    if ((rc = coop_admit(ctx, S, C))) return rc;
    const int slots = ctx->slots > 0 ? ctx->slots : S.max_batch;
    CoopBatch* oldest = nullptr;
    double t_old = 0.0;
    for (auto& B : C.batches)
        for (auto& I : B->in)
            if (!oldest || I.r->t_submit < t_old) {
                oldest = B.get();
                t_old = I.r->t_submit;
            }
    if (oldest && (rc = coop_cycle(ctx, S, *oldest, slots))) {
        // a failed cycle ends its requests (the others keep going)
        for (auto& I : oldest->in) coop_done(S, I.r, rc);
        oldest->in.clear();
        oldest->b.ds.clear();
    }
    C.batches.erase(std::remove_if(C.batches.begin(), C.batches.end(),
                                   [](const std::unique_ptr<CoopBatch>& B) { return B->in.empty(); }),
                    C.batches.end());
    return SSA_OK;
}

int serve_start(ssa_ctx* ctx) {
    if (ctx->srv.load(std::memory_order_acquire)) return SSA_OK;
    std::lock_guard<std::mutex> start_lock(ctx->srv_mu);
    if (ctx->srv.load(std::memory_order_acquire)) return SSA_OK;
    auto* S = new Server();
    int nw = 3;
    if (const char* e = std::getenv("SHSSA_SERVE_WORKERS")) nw = std::max(1, std::min(8, std::atoi(e)));
    for (int w = 0; w < nw; ++w) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            for (auto x : S->streams) (void)hipStreamDestroy(x);
            delete S;
            return fail(SSA_EDEVICE, "stream creation failed");
        }
        S->streams.push_back(s);
    }
    ctx->srv.store(S, std::memory_order_release);
    for (int w = 0; w < nw; ++w) S->workers.emplace_back(serve_worker, ctx, w);
    return SSA_OK;
}

// The request of a ticket (nullptr if unknown) and whether it is done.
std::shared_ptr<ServeReq> find_ticket(Server& S, uint64_t ticket, bool* done) {
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.reqs.find(ticket);
    if (it == S.reqs.end()) return nullptr;
    *done = it->second->done;
    return it->second;
}

// The cooperative server: a queue and its batches, no threads.
int coop_start(ssa_ctx* ctx) {
    if (ctx->srv.load(std::memory_order_acquire)) return SSA_OK;
    std::lock_guard<std::mutex> start_lock(ctx->srv_mu);
    if (ctx->srv.load(std::memory_order_acquire)) return SSA_OK;
    auto* S = new Server();
    S->coop = std::make_shared<CoopState>();
    ctx->srv.store(S, std::memory_order_release);
    return SSA_OK;
}

void serve_stop(ssa_ctx* ctx) {
    Server* S = ctx->srv;
    if (!S) return;
    if (S->coop) {
        // queued work of the batches first, then the batches (they refer to
        // the requests' handles), then the requests
        std::lock_guard<std::recursive_mutex> call(ctx->call_mu);
        (void)hipStreamSynchronize(ctx->st);
        S->coop->batches.clear();
        S->pending.clear();
        S->reqs.clear();
        ctx->srv = nullptr;
        delete S;
        return;
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    for (auto& t : S->workers) t.join();
    S->pending.clear();
    S->reqs.clear();   // frees the handles of requests never taken
    for (auto s : S->streams) {
        ctx->stage_drop(s);
        (void)hipStreamDestroy(s);
    }
    ctx->srv = nullptr;
    delete S;
}

// ---------------------------------------------------------------------------
// fixed device scratch of the allocation-free calls
// ---------------------------------------------------------------------------

// One array per GPU that the library runs on, held until the process ends.
// Host code never uses its name as an address (on the host it only names
// the symbol): scratch_init looks up each device's copy once, with that
// device current, and the calls pass that address to their kernels.
constexpr size_t kScratchBytes = 64u << 10;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, unsigned char*> g_scratch_ptr;   // device -> address of its scratch
}  // namespace

// Called by ssa_ctx_create with `device` current.
int scratch_init(int device) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_ptr.count(device)) return SSA_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(SSA_EDEVICE, "no address for the device scratch");
    g_scratch_ptr[device] = static_cast<unsigned char*>(p);
    return SSA_OK;
}

unsigned char* scratch_of(int device) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    return it == g_scratch_ptr.end() ? nullptr : it->second;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

namespace {
// Holds the context's call lock for one entry point (no lock for a null
// context; the entry point then fails its argument check).
struct CallLock {
    std::unique_lock<std::recursive_mutex> lk;
    explicit CallLock(ssa_ctx* c) {
        if (c) lk = std::unique_lock<std::recursive_mutex>(c->call_mu);
    }
};
}  // namespace

namespace {

// A one-dimensional request (window along the series, full box) whose
// natural transform row is longer than one workgroup's transforms hold.
bool long_series(const ssa_request& q) {
    const bool colv = q.ny == 1 && q.ly == 1 && q.lx > 1, rowv = q.nx == 1 && q.lx == 1 && q.ly > 1;
    if (!colv && !rowv) return false;
    if (q.wmask)
        for (long i = 0; i < (long)q.lx * q.ly; ++i)
            if (!q.wmask[i]) return false;
    const int n = colv ? q.nx : q.ny, l = colv ? q.lx : q.ly;
    if (l >= n) return false;
    return row_class(next_smooth((n + 1) / 2), q.precision == SSA_FP64) < 0;
}

// The segments' MSSA decomposition of a long series: segments of one
// power-of-two transform row S = B + L - 1 (8192 complex points in FP64,
// 16384 in FP32), the last one shorter.
int decompose_long_series(ssa_ctx* ctx, const ssa_request& q, ssa_decomp** out) {
    *out = nullptr;
    const bool colv = q.ny == 1;
    const int N = colv ? q.nx : q.ny, L = colv ? q.lx : q.ly;
    const int S = 2 * (q.precision == SSA_FP64 ? 8192 : 16384);
    if (2 * L > S)
        return fail(SSA_EINVAL, "series longer than one transform row with a window of more than half a segment");
    const int B = S - L + 1, K0 = N - L + 1;
    const int s = (K0 + B - 1) / B, nmax = B + L - 1;
    std::vector<double> xs(N);
    for (int t = 0; t < N; ++t) xs[t] = (q.mask && !q.mask[t]) ? std::nan("") : q.x[t];
    std::vector<double> packed((size_t)nmax * s, std::nan(""));
    for (int p = 0; p < s; ++p) {
        const int len = std::min(nmax, N - p * B);
        for (int t = 0; t < len; ++t) packed[(size_t)t * s + p] = xs[(size_t)p * B + t];
    }
    ssa_request q2{packed.data(), nmax, s, nullptr, nullptr, L, 1, q.r, q.precision, q.seed};
    int st = SSA_OK;
    const int rc = decompose_many(ctx, 1, &q2, out, &st, false);
    if (*out) {
        auto& g = (*out)->seg;
        g.on = true;
        g.col = colv;
        g.N = N;
        g.L = L;
        g.B = B;
        g.s = s;
        g.nmax = nmax;
        g.x.swap(xs);
    }
    return rc ? rc : st;
}

// Sum over the segments of a packed array (nmax x s, row-major) onto the
// series: out[t] = sum_p a(t - p B, p), NaN terms skipped.
void seg_sum(const ssa_decomp::Seg& g, const double* a, double* out) {
    for (int t = 0; t < g.N; ++t) out[t] = 0.0;
    for (int p = 0; p < g.s; ++p)
        for (int u = 0; u < g.nmax && (long)p * g.B + u < g.N; ++u) {
            const double v = a[(size_t)u * g.s + p];
            if (!std::isnan(v)) out[(size_t)p * g.B + u] += v;
        }
}

}  // namespace

int ssa_ctx_profile(ssa_ctx* ctx, const char* kind) {
    if (!ctx) return fail(SSA_EINVAL, "ctx is NULL");
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->prof_kinds.clear();
    if (kind) {
        std::string all(kind), cur;
        for (char ch : all + ",") {
            if (ch == ',') {
                if (!cur.empty()) ctx->prof_kinds.push_back(cur);
                cur.clear();
            } else {
                cur += ch;
            }
        }
    }
    ctx->prof_seen.assign(ctx->prof_kinds.size(), 0);
    if (!ctx->prof_kinds.empty()) {
        if (!ctx->prof_ref) HIPCHK(hipEventCreate(&ctx->prof_ref));
        HIPCHK(hipEventRecord(ctx->prof_ref, ctx->st));
    }
    return SSA_OK;
}

int ssa_ctx_profile_every(ssa_ctx* ctx, int every) {
    if (!ctx) return fail(SSA_EINVAL, "ctx is NULL");
    if (every < 1) return fail(SSA_EINVAL, "every must be >= 1");
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->prof_every = every;
    return SSA_OK;
}

// Time during which at least one recorded launch of class kind (all classes
// for kind = NULL) was running, with the launch count and algorithmic bytes.
static int profile_sum(ssa_ctx* ctx, const char* kind, double* ms, long* launches, double* bytes) {
    const int want = kind ? ctx->prof_index(kind) : -1;
    if (kind && want < 0) return fail(SSA_EINVAL, "kernel class not recorded");
    // launches of concurrent streams may overlap: the time is the length of
    // the union of the recorded [start, end] intervals
    std::vector<std::pair<double, double>> iv;
    long n = 0;
    double by = 0.0;
    for (auto& sp : ctx->spans) {
        if (kind && sp.kind != want) continue;
        float a = 0.f, b = 0.f;
        HIPCHK(hipEventSynchronize(ctx->ev_pool[sp.e1]));
        HIPCHK(hipEventElapsedTime(&a, ctx->prof_ref, ctx->ev_pool[sp.e0]));
        HIPCHK(hipEventElapsedTime(&b, ctx->prof_ref, ctx->ev_pool[sp.e1]));
        iv.push_back({a, b});
        ++n;
        by += sp.bytes;
    }
    std::sort(iv.begin(), iv.end());
    double tot = 0.0, cs = 0.0, ce = -1e300;
    for (auto& x : iv) {
        if (x.first > ce) {
            if (ce > cs) tot += ce - cs;
            cs = x.first;
            ce = x.second;
        } else {
            ce = std::max(ce, x.second);
        }
    }
    if (ce > cs && !iv.empty()) tot += ce - cs;
    if (ms) *ms = tot;
    if (launches) *launches = n;
    if (bytes) *bytes = by;
    return SSA_OK;
}

int ssa_ctx_profile_read(ssa_ctx* ctx, double* ms, long* launches, double* bytes) {
    CallLock call(ctx);
    if (!ctx) return fail(SSA_EINVAL, "ctx is NULL");
    HIPCHK(hipStreamSynchronize(ctx->st));
    std::lock_guard<std::mutex> g(ctx->mu);
    int rc = profile_sum(ctx, nullptr, ms, launches, bytes);
    ctx->spans.clear();
    ctx->ev_next = 0;
    return rc;
}

int ssa_ctx_profile_launches(ssa_ctx* ctx, const char* kind, long* launches) {
    if (!ctx || !kind || !launches) return fail(SSA_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(ctx->mu);
    const int k = ctx->prof_index(kind);
    if (k < 0) return fail(SSA_EINVAL, "kernel class not recorded");
    *launches = ctx->prof_seen[k];
    return SSA_OK;
}

int ssa_ctx_profile_read_kind(ssa_ctx* ctx, const char* kind, double* ms, long* launches, double* bytes) {
    CallLock call(ctx);
    if (!ctx || !kind) return fail(SSA_EINVAL, "NULL argument");
    HIPCHK(hipStreamSynchronize(ctx->st));
    std::lock_guard<std::mutex> g(ctx->mu);
    return profile_sum(ctx, kind, ms, launches, bytes);
}

int ssa_ctx_create(int device, size_t mem_budget, const char* tune_cache, ssa_ctx** out) {
    if (!out) return fail(SSA_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(SSA_EDEVICE, "no HIP device");
    if (device < 0 || device >= ndev) return fail(SSA_EINVAL, "device out of range");
    HIPCHK(hipSetDevice(device));
    if (int rc = scratch_init(device)) return rc;
    auto* c = new ssa_ctx();
    c->device = device;
    c->budget = mem_budget;
    c->len_tune = std::getenv("SHSSA_LEN_TUNE") != nullptr;
    if (hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return fail(SSA_EDEVICE, "hipStreamCreate failed");
    }
    c->own = true;
    if (tune_cache && *tune_cache) {
        c->tune_path = tune_cache;
        std::lock_guard<std::mutex> g(c->tune_mu);
        c->tune_load();
    }
    *out = c;
    return SSA_OK;
}

void ssa_ctx_destroy(ssa_ctx* ctx) {
    if (!ctx) return;
    serve_stop(ctx);
    bool now = false;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        ctx->closing = true;
        now = ctx->refs == 0;
    }
    if (now) ctx_release(ctx);
}

int ssa_ctx_set_stream(ssa_ctx* ctx, void* stream) {
    CallLock call(ctx);
    if (!ctx) return fail(SSA_EINVAL, "ctx is NULL");
    HIPCHK(hipStreamSynchronize(ctx->st));
    if (ctx->own) (void)hipStreamDestroy(ctx->st);
    ctx->own = false;
    ctx->st = static_cast<hipStream_t>(stream);
    return SSA_OK;
}

int ssa_ctx_set_slots(ssa_ctx* ctx, int slots) {
    CallLock call(ctx);
    if (!ctx) return fail(SSA_EINVAL, "ctx is NULL");
    if (slots < 0) return fail(SSA_EINVAL, "slots must be >= 0");
    ctx->slots = slots;
    return SSA_OK;
}

int ssa_ctx_sync(ssa_ctx* ctx) {
    CallLock call(ctx);
    if (!ctx) return fail(SSA_EINVAL, "ctx is NULL");
    HIPCHK(hipStreamSynchronize(ctx->st));
    return SSA_OK;
}

int ssa_decompose_batch(ssa_ctx* ctx, int n, const ssa_request* reqs, ssa_decomp** out, int* status) {
    CallLock call(ctx);
    return decompose_many(ctx, n, reqs, out, status, false);
}

int ssa_decompose_batch_dev(ssa_ctx* ctx, int n, const ssa_request* reqs, ssa_decomp** out, int* status) {
    CallLock call(ctx);
    return decompose_many(ctx, n, reqs, out, status, true);
}

int ssa_decompose(ssa_ctx* ctx, const double* x, int nx, int ny, const uint8_t* mask, const uint8_t* wmask,
                  int lx, int ly, int r, int precision, ssa_decomp** out) {
    CallLock call(ctx);
    if (!out) return fail(SSA_EINVAL, "out is NULL");
    ssa_request q{x, nx, ny, mask, wmask, lx, ly, r, precision, 0x5eedULL};
    if (ctx && x && long_series(q)) return decompose_long_series(ctx, q, out);
    int st = SSA_OK;
    int rc = decompose_many(ctx, 1, &q, out, &st, false);
    return rc ? rc : st;
}

int ssa_decompose_eigen(ssa_ctx* ctx, const double* x, int nx, int ny, const uint8_t* mask, const uint8_t* wmask,
                        int lx, int ly, int r, ssa_decomp** out) {
    CallLock call(ctx);
    if (!out) return fail(SSA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctx) return fail(SSA_EINVAL, "context is NULL");
    ssa_request q{x, nx, ny, mask, wmask, lx, ly, r, SSA_FP64, 0x5eedULL};
    g_tables_ctx = ctx;
    TableScope tables(ctx, ctx->st);
    std::unique_ptr<ssa_decomp> d(new ssa_decomp());
    int rc = plan_request(ctx, q, d.get());
    if (rc) return rc;
    if (d->L > kEigMaxL) return fail(SSA_EINVAL, "eigen method needs a window of at most 4096 cells");
    if ((rc = upload_request(q, d.get(), false, ctx->st))) return rc;
    d->eigen = true;
    std::vector<int> st;
    run_planned(ctx, {d.get()}, ctx->st, st);
    if (st.empty() || st[0] != SSA_OK) return st.empty() ? fail(SSA_EINVAL, "no decomposition") : st[0];
    (void)seal_handle(d.get());
    *out = d.release();
    return SSA_OK;
}

int ssa_decompose_multi(ssa_ctx* ctx, const double* const* series, const int* len, int s, int L, int r,
                        int precision, ssa_decomp** out) {
    CallLock call(ctx);
    if (!out) return fail(SSA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!series || !len || s <= 0) return fail(SSA_EINVAL, "no series");
    int nmax = 0, nmin = 1 << 30;
    for (int p = 0; p < s; ++p) {
        if (len[p] <= 0 || !series[p]) return fail(SSA_EINVAL, "empty series");
        nmax = std::max(nmax, len[p]);
        nmin = std::min(nmin, len[p]);
    }
    if (!(L > 1 && L < nmin)) return fail(SSA_EINVAL, "window must satisfy 1 < L < min N_p");
    // 2D packing: max N_p x s array, column p = series p, NaN below its end
    std::vector<double> x((size_t)nmax * s, std::nan(""));
    for (int p = 0; p < s; ++p)
        for (int t = 0; t < len[p]; ++t) x[(size_t)t * s + p] = series[p][t];
    ssa_request q{x.data(), nmax, s, nullptr, nullptr, L, 1, r, precision, 0x5eedULL};
    int st = SSA_OK;
    int rc = decompose_many(ctx, 1, &q, out, &st, false);
    return rc ? rc : st;
}

int ssa_decompose_m2d(ssa_ctx* ctx, const double* const* images, const int* nx, const int* ny, int s,
                      const uint8_t* wmask, int lx, int ly, int r, int precision, int* col_off, ssa_decomp** out) {
    CallLock call(ctx);
    if (!out) return fail(SSA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!images || !nx || !ny || s <= 0) return fail(SSA_EINVAL, "no images");
    if (lx <= 0 || ly <= 0) return fail(SSA_EINVAL, "sizes must be positive");
    // one separator column for a full window; ly - 1 for a shaped one, whose
    // holes could otherwise let a window reach across a single column
    const int sep = wmask ? std::max(1, ly - 1) : 1;
    int nxmax = 0;
    long width = (long)sep * (s - 1);
    for (int p = 0; p < s; ++p) {
        if (nx[p] <= 0 || ny[p] <= 0 || !images[p]) return fail(SSA_EINVAL, "empty image");
        nxmax = std::max(nxmax, nx[p]);
        width += ny[p];
    }
    if ((double)nxmax * (double)width > 2e9) return fail(SSA_EINVAL, "packed array too large");
    std::vector<double> x((size_t)nxmax * width, std::nan(""));
    long c = 0;
    for (int p = 0; p < s; ++p) {
        if (col_off) col_off[p] = (int)c;
        for (int i = 0; i < nx[p]; ++i)
            std::memcpy(&x[(size_t)i * width + c], images[p] + (size_t)i * ny[p], (size_t)ny[p] * sizeof(double));
        c += ny[p] + sep;
    }
    ssa_request q{x.data(), nxmax, (int)width, nullptr, wmask, lx, ly, r, precision, 0x5eedULL};
    int st = SSA_OK;
    int rc = decompose_many(ctx, 1, &q, out, &st, false);
    return rc ? rc : st;
}

int ssa_decompose_mosaic(ssa_ctx* ctx, const double* const* series, int s, int t, const int* Ls, const int* Ks,
                         int r, int precision, int* col_off, ssa_decomp** out) {
    CallLock call(ctx);
    if (!out) return fail(SSA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!series || !Ls || !Ks || s <= 0 || t <= 0) return fail(SSA_EINVAL, "no blocks");
    int Lm = 0;
    for (int i = 0; i < s; ++i) {
        if (Ls[i] <= 0) return fail(SSA_EINVAL, "block row sizes L_i must be positive");
        Lm = std::max(Lm, Ls[i]);
    }
    for (int j = 0; j < t; ++j)
        if (Ks[j] <= 0) return fail(SSA_EINVAL, "block column sizes K_j must be positive");
    for (int e = 0; e < s * t; ++e)
        if (!series[e]) return fail(SSA_EINVAL, "NULL series");
    // block column j from column off[j]: Lm + K_j - 1 columns, then one NaN
    // column (none after the last)
    std::vector<long> off(t);
    long width = 0;
    for (int j = 0; j < t; ++j) {
        off[j] = width;
        width += (long)Lm + Ks[j];
    }
    width -= 1;
    if ((double)s * (double)width > 2e9) return fail(SSA_EINVAL, "packed array too large");
    std::vector<double> x((size_t)s * width, std::nan(""));
    for (int i = 0; i < s; ++i)
        for (int j = 0; j < t; ++j)
            std::memcpy(&x[(size_t)i * width + off[j]], series[(size_t)i * t + j],
                        (size_t)(Ls[i] + Ks[j] - 1) * sizeof(double));
    // window: s rows, row i its first L_i cells
    std::vector<uint8_t> wm((size_t)s * Lm, 0);
    for (int i = 0; i < s; ++i) std::memset(&wm[(size_t)i * Lm], 1, (size_t)Ls[i]);
    if (col_off)
        for (int j = 0; j < t; ++j) col_off[j] = (int)off[j];
    ssa_request q{x.data(), s, (int)width, nullptr, wm.data(), s, Lm, r, precision, 0x5eedULL};
    int st = SSA_OK;
    int rc = decompose_many(ctx, 1, &q, out, &st, false);
    return rc ? rc : st;
}

int ssa_get_dims(const ssa_decomp* d, int* lx, int* ly, int* kx, int* ky, long* L, long* K, int* r, int* nx,
                 int* ny) {
    if (!d) return fail(SSA_EINVAL, "handle is NULL");
    if (d->seg.on) {   // the series' geometry (N x 1 or 1 x N)
        const auto& g = d->seg;
        const int K0 = g.N - g.L + 1;
        if (lx) *lx = g.col ? g.L : 1;
        if (ly) *ly = g.col ? 1 : g.L;
        if (kx) *kx = g.col ? K0 : 1;
        if (ky) *ky = g.col ? 1 : K0;
        if (L) *L = d->L;
        if (K) *K = d->K;
        if (r) *r = d->r;
        if (nx) *nx = g.col ? g.N : 1;
        if (ny) *ny = g.col ? 1 : g.N;
        return SSA_OK;
    }
    if (lx) *lx = d->lx;
    if (ly) *ly = d->ly;
    if (kx) *kx = d->kx;
    if (ky) *ky = d->ky;
    if (L) *L = d->L;
    if (K) *K = d->K;
    if (r) *r = d->r;
    if (nx) *nx = d->nx;
    if (ny) *ny = d->ny;
    return SSA_OK;
}

int ssa_get_sigma(const ssa_decomp* dc, double* sigma) {
    CallLock call(dc ? dc->ctx : nullptr);
    auto* d = const_cast<ssa_decomp*>(dc);
    if (!d || !sigma) return fail(SSA_EINVAL, "NULL argument");
    if (!d->decomposed) return fail(SSA_ESTATE, "not decomposed");
    if (!d->sigma_ready) {
        int rc;
        if ((rc = wait_handle(d))) return rc;
        d->sigma_h.resize(d->r);
        HIPCHK(hipMemcpy(d->sigma_h.data(), d->sigma, d->r * sizeof(double), hipMemcpyDeviceToHost));
        d->sigma_ready = true;
    }
    std::memcpy(sigma, d->sigma_h.data(), d->r * sizeof(double));
    return SSA_OK;
}

static int vectors_raw(ssa_decomp* d, double* U, double* V);

int ssa_get_vectors(const ssa_decomp* dc, double* U, double* V) {
    CallLock call(dc ? dc->ctx : nullptr);
    auto* d = const_cast<ssa_decomp*>(dc);
    if (!d) return fail(SSA_EINVAL, "handle is NULL");
    if (!d->seg.on) return vectors_raw(d, U, V);
    // segments: U as it is; V of the series = the segments' V side by side
    const auto& g = d->seg;
    std::vector<double> vm;
    if (V) vm.resize((size_t)d->kx * d->ky * d->r);
    int rc = vectors_raw(d, U, V ? vm.data() : nullptr);
    if (rc || !V) return rc;
    const long K0 = g.N - g.L + 1, box = (long)d->kx * d->ky;
    for (int c = 0; c < d->r; ++c)
        for (long k = 0; k < K0; ++k) {
            const int p = (int)(k / g.B), u = (int)(k % g.B);
            V[(long)c * K0 + k] = vm[(size_t)c * box + (size_t)u * g.s + p];
        }
    return SSA_OK;
}

static int vectors_raw(ssa_decomp* d, double* U, double* V) {
    if (!d->decomposed) return fail(SSA_ESTATE, "not decomposed");
    int rc;
    if ((rc = wait_handle(d))) return rc;
    if (U) {
        std::vector<double> u((size_t)d->L * d->r);
        HIPCHK(hipMemcpy(u.data(), d->U, u.size() * 8, hipMemcpyDeviceToHost));
        const long box = (long)d->lx * d->ly;
        std::fill(U, U + box * d->r, std::nan(""));
        const uint8_t* m = d->L == (long)d->LA * d->LB ? nullptr : d->lmask_h.data();
        walk_set(d, d->LA, d->LB, m, [&](long idx, int i, int j) {
            for (int c = 0; c < d->r; ++c) U[c * box + (long)i * d->ly + j] = u[(size_t)c * d->L + idx];
        });
    }
    if (V) {
        if ((rc = fetch_kmask(d))) return rc;
        std::vector<double> v((size_t)d->K * d->r);
        HIPCHK(hipMemcpy(v.data(), d->V, v.size() * 8, hipMemcpyDeviceToHost));
        const long box = (long)d->kx * d->ky;
        std::fill(V, V + box * d->r, std::nan(""));
        walk_set(d, d->KA, d->KB, d->kmask_h.data(), [&](long idx, int i, int j) {
            for (int c = 0; c < d->r; ++c) V[c * box + (long)i * d->ky + j] = v[(size_t)c * d->K + idx];
        });
    }
    return SSA_OK;
}

int ssa_get_vectors_lex(const ssa_decomp* dc, double* U, double* V) {
    CallLock call(dc ? dc->ctx : nullptr);
    auto* d = const_cast<ssa_decomp*>(dc);
    if (!d) return fail(SSA_EINVAL, "handle is NULL");
    const long lb = (long)d->lx * d->ly, kb = (long)d->kx * d->ky;
    std::vector<double> gu(lb * d->r), gv(kb * d->r);
    // (for a segmented series the segments' lexicographic order of K is the
    // series' order: segment by segment, origins in order within each)
    int rc = vectors_raw(d, gu.data(), V ? gv.data() : nullptr);
    if (rc) return rc;
    // lexicographic = column-major over the caller's box (row index fastest)
    auto pack = [&](const std::vector<double>& g, int bx, int by, long cnt, double* out) {
        const long box = (long)bx * by;
        for (int c = 0; c < d->r; ++c) {
            long k = 0;
            for (int j = 0; j < by; ++j)
                for (int i = 0; i < bx; ++i) {
                    const double v = g[c * box + (long)i * by + j];
                    if (!std::isnan(v) || false) out[(long)c * cnt + k++] = v;
                }
        }
    };
    if (U) {
        // window cells can hold any value; walk the mask instead of NaN tests
        const long box = lb;
        for (int c = 0; c < d->r; ++c) {
            long k = 0;
            for (int j = 0; j < d->ly; ++j)
                for (int i = 0; i < d->lx; ++i) {
                    const int a = d->tr ? j : i, b = d->tr ? i : j;
                    if (d->lmask_h[(size_t)a * d->LB + b]) U[(long)c * d->L + k++] = gu[c * box + (long)i * d->ly + j];
                }
        }
    }
    if (V) {
        for (int c = 0; c < d->r; ++c) {
            long k = 0;
            for (int j = 0; j < d->ky; ++j)
                for (int i = 0; i < d->kx; ++i) {
                    const int a = d->tr ? j : i, b = d->tr ? i : j;
                    if (d->kmask_h[(size_t)a * d->KB + b]) V[(long)c * d->K + k++] = gv[c * kb + (long)i * d->ky + j];
                }
        }
    }
    (void)pack;
    return SSA_OK;
}

static int weights_raw(ssa_decomp* d, double* w);

int ssa_get_weights(const ssa_decomp* dc, double* w) {
    CallLock call(dc ? dc->ctx : nullptr);
    auto* d = const_cast<ssa_decomp*>(dc);
    if (!d || !w) return fail(SSA_EINVAL, "NULL argument");
    if (!d->seg.on) return weights_raw(d, w);
    std::vector<double> wm((size_t)d->nx * d->ny);
    const int rc = weights_raw(d, wm.data());
    if (!rc) seg_sum(d->seg, wm.data(), w);
    return rc;
}

static int weights_raw(ssa_decomp* d, double* w) {
    int rc;
    if ((rc = wait_handle(d))) return rc;
    const long n = (long)d->A * d->B;
    if (!d->tr) {
        HIPCHK(hipMemcpy(w, d->W, n * 8, hipMemcpyDeviceToHost));
    } else {
        std::vector<double> t(n);
        HIPCHK(hipMemcpy(t.data(), d->W, n * 8, hipMemcpyDeviceToHost));
        for (int a = 0; a < d->A; ++a)
            for (int b = 0; b < d->B; ++b) w[(long)b * d->A + a] = t[(long)a * d->B + b];
    }
    return SSA_OK;
}

static int check_groups(const ssa_decomp* d, const int* gp, const int* gi, int ng) {
    if (ng <= 0 || !gp || !gi) return fail(SSA_EINVAL, "no groups");
    if (gp[0] != 0) return fail(SSA_EINVAL, "grp_ptr[0] must be 0");
    for (int g = 0; g < ng; ++g)
        if (gp[g + 1] < gp[g]) return fail(SSA_EINVAL, "grp_ptr must be non-decreasing");
    for (int k = 0; k < gp[ng]; ++k)
        if (gi[k] < 0 || gi[k] >= d->r) return fail(SSA_EINVAL, "component id out of range");
    if (ng > d->r) return fail(SSA_EINVAL, "more groups than components");
    return SSA_OK;
}

static int reconstruct_raw(ssa_decomp* d, const int* gp, const int* gi, int ng, double* out);

int ssa_reconstruct(ssa_decomp* d, const int* gp, const int* gi, int ng, double* out) {
    CallLock call(d ? d->ctx : nullptr);
    if (!d || !out) return fail(SSA_EINVAL, "NULL argument");
    if (!d->seg.on) return reconstruct_raw(d, gp, gi, ng, out);
    if (!d->decomposed) return fail(SSA_ESTATE, "not decomposed");
    int rc = check_groups(d, gp, gi, ng);
    if (rc) return rc;
    // segments: x~_t = sum_p W_p x~_p / sum_p W_p over the segments holding t
    const auto& g = d->seg;
    const size_t np = (size_t)d->nx * d->ny;
    std::vector<double> wm(np), rm(np * ng), num(g.N), den(g.N), wr(np);
    if ((rc = weights_raw(d, wm.data())) || (rc = reconstruct_raw(d, gp, gi, ng, rm.data()))) return rc;
    seg_sum(g, wm.data(), den.data());
    for (int k = 0; k < ng; ++k) {
        for (size_t e = 0; e < np; ++e) wr[e] = wm[e] > 0 ? wm[e] * rm[(size_t)k * np + e] : std::nan("");
        seg_sum(g, wr.data(), num.data());
        for (int t = 0; t < g.N; ++t) out[(size_t)k * g.N + t] = den[t] > 0 ? num[t] / den[t] : std::nan("");
    }
    return SSA_OK;
}

static int reconstruct_raw(ssa_decomp* d, const int* gp, const int* gi, int ng, double* out) {
    if (!d->decomposed) return fail(SSA_ESTATE, "not decomposed");
    int rc = check_groups(d, gp, gi, ng);
    if (rc) return rc;
    const long n = (long)d->A * d->B;
    g_tables_ctx = d->ctx;
    TableScope tables(d->ctx, d->ctx->st);
    DevVec rbuf;   // from the pool: no device-wide synchronisation of hipFree
    if ((rc = rbuf.reserve((size_t)n * ng * 8))) return rc;
    double* buf = rbuf.as<double>();
    Batch b(d->ctx);
    b.ds = {d};
    b.f64 = d->f64;
    b.rowfam = d->rowfam;
    b.cls = row_word(d->nh, d->f64);
    b.set_col(d->ctx->tile_for(d->f64, d->MA));
    rc = run_reconstruct(b, std::vector<int>(gp, gp + ng + 1), std::vector<int>(gi, gi + gp[ng]), {buf});
    if (!rc && hipStreamSynchronize(b.st) != hipSuccess) rc = fail(SSA_EDEVICE, "reconstruction");
    if (!rc) {
        if (!d->tr) {
            if (hipMemcpy(out, buf, n * ng * 8, hipMemcpyDeviceToHost) != hipSuccess) rc = fail(SSA_EDEVICE, "copy");
        } else {
            std::vector<double> t(n * ng);
            if (hipMemcpy(t.data(), buf, n * ng * 8, hipMemcpyDeviceToHost) != hipSuccess) rc = fail(SSA_EDEVICE, "copy");
            for (int g = 0; g < ng; ++g)
                for (int a = 0; a < d->A; ++a)
                    for (int bb = 0; bb < d->B; ++bb)
                        out[g * n + (long)bb * d->A + a] = t[g * n + (long)a * d->B + bb];
        }
    }
    return rc;
}

int ssa_wcor(ssa_decomp* d, const int* gp, const int* gi, int ng, double* rho, double* contrib) {
    CallLock call(d ? d->ctx : nullptr);
    if (!d || !rho) return fail(SSA_EINVAL, "NULL argument");
    if (!d->decomposed) return fail(SSA_ESTATE, "not decomposed");
    int rc = check_groups(d, gp, gi, ng);
    if (rc || (rc = wait_handle(d))) return rc;
    if (d->seg.on) {
        // segmented series: the same weighted inner products over the
        // series' reconstructions and weights (host, O(ng^2 N))
        const auto& g = d->seg;
        std::vector<double> rec((size_t)ng * g.N), w(g.N);
        if ((rc = ssa_reconstruct(d, gp, gi, ng, rec.data())) || (rc = ssa_get_weights(d, w.data()))) return rc;
        auto dot = [&](const double* a, const double* b) {
            double acc = 0.0;
            for (int t = 0; t < g.N; ++t)
                if (w[t] > 0 && !std::isnan(a[t]) && !std::isnan(b[t])) acc += w[t] * a[t] * b[t];
            return acc;
        };
        const double xx = dot(g.x.data(), g.x.data());
        std::vector<double> nn(ng);
        for (int a = 0; a < ng; ++a) nn[a] = dot(&rec[(size_t)a * g.N], &rec[(size_t)a * g.N]);
        for (int a = 0; a < ng; ++a) {
            for (int c = 0; c < ng; ++c) {
                const double den = std::sqrt(nn[a] * nn[c]);
                rho[(size_t)a * ng + c] =
                    den > 0 ? (a == c ? nn[a] : dot(&rec[(size_t)a * g.N], &rec[(size_t)c * g.N])) / den : 0.0;
            }
            if (contrib) contrib[a] = xx > 0 ? nn[a] / xx : 0.0;
        }
        return SSA_OK;
    }
    g_tables_ctx = d->ctx;
    TableScope tables(d->ctx, d->ctx->st);
    Batch b(d->ctx);
    b.ds = {d};
    b.f64 = d->f64;
    b.rowfam = d->rowfam;
    b.cls = row_word(d->nh, d->f64);
    b.set_col(d->ctx->tile_for(d->f64, d->MA));
    const long n = (long)d->A * d->B;
    // the groups' reconstructions (internal orientation) and the cleaned
    // input (equal to x on the covered set) are the arrays of the Gram
    DevVec rec, part, out;
    if ((rc = rec.reserve((size_t)ng * n * sizeof(double)))) return rc;
    if ((rc = run_reconstruct(b, std::vector<int>(gp, gp + ng + 1), std::vector<int>(gi, gi + gp[ng]),
                              {rec.as<double>()})))
        return rc;
    const int narr = ng + 1;
    std::vector<const double*> arr;
    for (int g = 0; g < ng; ++g) arr.push_back(rec.as<double>() + (long)g * n);
    arr.push_back(d->xc);
    DevVec darr;
    if ((rc = darr.put(arr, b.st))) return rc;
    const int tiles = wgram_tiles(narr);
    // about 1024 workgroups in all, each with at least 512 cells
    const int nchunk = (int)std::max<long>(1, std::min<long>(1024 / tiles + 1, n / 512));
    if ((rc = part.reserve((size_t)tiles * 256 * nchunk * sizeof(double))) ||
        (rc = out.reserve((size_t)tiles * 256 * sizeof(double))))
        return rc;
    {
        // algorithmic bytes: every array and the weights read once
        ProfSpan p(b.ctx, "wgram", b.st, [&] { return (double)(narr + 1) * n * sizeof(double); });
        launch_wgram(b.st, darr.as<const double*>(), narr, d->W, n, nchunk, part.as<double>(), out.as<double>());
    }
    HIPCHK(hipGetLastError());
    std::vector<double> t((size_t)tiles * 256);
    HIPCHK(hipMemcpyAsync(t.data(), out.p, t.size() * sizeof(double), hipMemcpyDeviceToHost, b.st));
    HIPCHK(hipStreamSynchronize(b.st));
    // Gram matrix from the tiles (the entry with i <= j on diagonal tiles)
    std::vector<double> G((size_t)narr * narr, 0.0);
    const int nb = (narr + 15) / 16;
    int k = 0;
    for (int ib = 0; ib < nb; ++ib)
        for (int jb = ib; jb < nb; ++jb, ++k)
            for (int i = 0; i < 16; ++i)
                for (int j = 0; j < 16; ++j) {
                    const int a = 16 * ib + i, c = 16 * jb + j;
                    if (a >= narr || c >= narr || (ib == jb && j < i)) continue;
                    const double v = t[(size_t)k * 256 + 16 * i + j];
                    G[(size_t)a * narr + c] = G[(size_t)c * narr + a] = v;
                }
    const double xx = G[(size_t)ng * narr + ng];
    for (int a = 0; a < ng; ++a) {
        for (int c = 0; c < ng; ++c) {
            const double den = std::sqrt(G[(size_t)a * narr + a] * G[(size_t)c * narr + c]);
            rho[(size_t)a * ng + c] = den > 0 ? G[(size_t)a * narr + c] / den : 0.0;
        }
        if (contrib) contrib[a] = xx > 0 ? G[(size_t)a * narr + a] / xx : 0.0;
    }
    return SSA_OK;
}

// max_ij |(Y^T Y)_ij - delta_ij| over the r columns Y[:, c] = y + c * n of
// a device array (the Gram matrix on the matrix cores, unit weights),
// queued on b's stream; the caller holds the context's call lock and a
// table scope.
static int gram_deviation(Batch& b, const double* y, long n, int r, double* dev) {
    int rc;
    std::vector<const double*> arr;
    for (int c = 0; c < r; ++c) arr.push_back(y + (long)c * n);
    DevVec darr, part, out;
    if ((rc = darr.put(arr, b.st))) return rc;
    const int tiles = wgram_tiles(r);
    const int nchunk = (int)std::max<long>(1, std::min<long>(1024 / tiles + 1, n / 512));
    if ((rc = part.reserve((size_t)tiles * 256 * nchunk * sizeof(double))) ||
        (rc = out.reserve((size_t)tiles * 256 * sizeof(double))))
        return rc;
    launch_wgram(b.st, darr.as<const double*>(), r, nullptr, n, nchunk, part.as<double>(), out.as<double>());
    HIPCHK(hipGetLastError());
    std::vector<double> t((size_t)tiles * 256);
    HIPCHK(hipMemcpyAsync(t.data(), out.p, t.size() * sizeof(double), hipMemcpyDeviceToHost, b.st));
    HIPCHK(hipStreamSynchronize(b.st));
    const int nb = (r + 15) / 16;
    double m = 0.0;
    int k = 0;
    for (int ib = 0; ib < nb; ++ib)
        for (int jb = ib; jb < nb; ++jb, ++k)
            for (int i = 0; i < 16; ++i)
                for (int j = 0; j < 16; ++j) {
                    const int a = 16 * ib + i, c = 16 * jb + j;
                    if (a >= r || c >= r || (ib == jb && j < i)) continue;
                    const double v = t[(size_t)k * 256 + 16 * i + j] - (a == c ? 1.0 : 0.0);
                    m = std::max(m, std::fabs(v));
                }
    *dev = m;
    return SSA_OK;
}

int ssa_orthogonality(ssa_decomp* d, double* orth_u, double* orth_v) {
    CallLock call(d ? d->ctx : nullptr);
    if (!d || !orth_u || !orth_v) return fail(SSA_EINVAL, "NULL argument");
    if (!d->decomposed) return fail(SSA_ESTATE, "not decomposed");
    int rc;
    if ((rc = wait_handle(d))) return rc;
    g_tables_ctx = d->ctx;
    TableScope tables(d->ctx, d->ctx->st);
    Batch b(d->ctx);
    if ((rc = gram_deviation(b, d->U, d->L, d->r, orth_u))) return rc;
    return gram_deviation(b, d->V, d->K, d->r, orth_v);
}

int ssa_rforecast(ssa_decomp* d, const int* grp, int ng, int h, double* out, int* nseries) {
    CallLock call(d ? d->ctx : nullptr);
    if (d && d->seg.on)
        return fail(SSA_EINVAL, "forecasts of a series decomposed in segments (longer than one transform row) are not supported");
    if (!d) return fail(SSA_EINVAL, "handle is NULL");
    if (!d->rowfam) return fail(SSA_EINVAL, "recurrent forecast needs a window one row or column wide");
    if (d->L != (long)d->LB) return fail(SSA_EINVAL, "recurrent forecast needs a window without mask");
    if (nseries) *nseries = d->A;
    if (!out) return SSA_OK;
    if (!d->decomposed) return fail(SSA_ESTATE, "not decomposed");
    if (!grp || ng < 1 || h < 1) return fail(SSA_EINVAL, "bad group or horizon");
    for (int k = 0; k < ng; ++k)
        if (grp[k] < 0 || grp[k] >= d->r) return fail(SSA_EINVAL, "component id out of range");
    int rc;
    if ((rc = wait_handle(d))) return rc;
    g_tables_ctx = d->ctx;
    TableScope tables(d->ctx, d->ctx->st);
    Batch b(d->ctx);
    b.ds = {d};
    b.f64 = d->f64;
    b.rowfam = d->rowfam;
    b.cls = row_word(d->nh, d->f64);
    b.set_col(d->ctx->tile_for(d->f64, d->MA));
    const long n = (long)d->A * d->B;
    const long L1 = d->L - 1;
    std::vector<int> g(grp, grp + ng);
    DevVec rec, R, flag, buf, outd, dg;
    if ((rc = rec.reserve((size_t)n * sizeof(double))) ||
        (rc = run_reconstruct(b, std::vector<int>{0, ng}, g, {rec.as<double>()})))
        return rc;
    if ((rc = dg.put(g, b.st)) || (rc = R.reserve((size_t)std::max<long>(L1, 1) * sizeof(double))) ||
        (rc = flag.reserve(sizeof(int))) || (rc = buf.reserve((size_t)d->A * (L1 + h) * sizeof(double))) ||
        (rc = outd.reserve((size_t)d->A * h * sizeof(double))))
        return rc;
    launch_rforecast(b.st, d->U, d->L, dg.as<int>(), ng, R.as<double>(), flag.as<int>(), rec.as<double>(), d->W,
                     d->A, d->B, h, buf.as<double>(), outd.as<double>());
    HIPCHK(hipGetLastError());
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, flag.p, sizeof(int), hipMemcpyDeviceToHost, b.st));
    HIPCHK(hipMemcpyAsync(out, outd.p, (size_t)d->A * h * sizeof(double), hipMemcpyDeviceToHost, b.st));
    HIPCHK(hipStreamSynchronize(b.st));
    if (bad) return fail(SSA_EINVAL, "no recurrent forecast: the group's last coordinates have nu^2 >= 1");
    return SSA_OK;
}

int ssa_vforecast(ssa_decomp* d, const int* grp, int ng, int h, double* out, int* nseries) {
    CallLock call(d ? d->ctx : nullptr);
    if (d && d->seg.on)
        return fail(SSA_EINVAL, "forecasts of a series decomposed in segments (longer than one transform row) are not supported");
    if (!d) return fail(SSA_EINVAL, "handle is NULL");
    if (!d->rowfam) return fail(SSA_EINVAL, "vector forecast needs a window one row or column wide");
    if (d->L != (long)d->LB) return fail(SSA_EINVAL, "vector forecast needs a window without mask");
    if (nseries) *nseries = d->A;
    if (!out) return SSA_OK;
    if (!d->decomposed) return fail(SSA_ESTATE, "not decomposed");
    if (!grp || ng < 1 || h < 1) return fail(SSA_EINVAL, "bad group or horizon");
    if (ng > kVfMaxGroup) return fail(SSA_EINVAL, "vector forecast group larger than 64 components");
    for (int k = 0; k < ng; ++k)
        if (grp[k] < 0 || grp[k] >= d->r) return fail(SSA_EINVAL, "component id out of range");
    int rc;
    if ((rc = wait_handle(d))) return rc;
    g_tables_ctx = d->ctx;
    TableScope tables(d->ctx, d->ctx->st);
    hipStream_t st = d->ctx->st;
    const long E = (long)h + d->L - 1;
    std::vector<int> g(grp, grp + ng);
    DevVec dg, M, flag, wbuf, outd;
    if ((rc = dg.put(g, st)) || (rc = flag.put(std::vector<int>{0, 0}, st)) ||
        (rc = M.reserve((size_t)ng * ng * sizeof(double))) ||
        (rc = wbuf.reserve((size_t)d->A * E * ng * sizeof(double))) ||
        (rc = outd.reserve((size_t)d->A * h * sizeof(double))))
        return rc;
    {
        // algorithmic bytes: the group's U columns and the coefficient vectors
        // written and read once per row, the forecasts written
        ProfSpan p(d->ctx, "vforecast", st, [&] {
            return 8.0 * ((double)ng * d->L + 2.0 * d->A * E * ng + (double)d->A * h);
        });
        launch_vforecast(st, d->U, d->L, d->V, d->K, d->sigma, dg.as<int>(), ng, M.as<double>(), d->krow, d->kmask,
                         d->KB, d->W, d->A, d->B, h, wbuf.as<double>(), outd.as<double>(), flag.as<int>());
    }
    HIPCHK(hipGetLastError());
    int bad[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(bad, flag.p, sizeof(bad), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(out, outd.p, (size_t)d->A * h * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (bad[1]) return fail(SSA_EINVAL, "no vector forecast: the group's last coordinates have nu^2 >= 1");
    if (bad[0]) return fail(SSA_EINVAL, "no vector forecast: a series' last lagged vector misses its last value");
    return SSA_OK;
}

int ssa_extend(ssa_decomp* d, int r_new) {
    CallLock call(d ? d->ctx : nullptr);
    if (!d) return fail(SSA_EINVAL, "handle is NULL");
    if (!d->decomposed || d->status != SSA_OK) return fail(SSA_ESTATE, "not decomposed");
    if (r_new <= d->r) return SSA_OK;
    if (r_new >= std::min(d->L, d->K)) return fail(SSA_ERANK, "r must be < min(L, K)");
    if (r_new > kMaxRank) return fail(SSA_ERANK, "r must be <= 120 (the basis holds 128 vectors)");
    int rc;
    if ((rc = wait_handle(d))) return rc;
    g_tables_ctx = d->ctx;
    TableScope tables(d->ctx, d->ctx->st);
    Batch b(d->ctx);
    b.ds = {d};
    b.f64 = d->f64;
    b.rowfam = d->rowfam;
    b.cls = row_word(d->nh, d->f64);
    b.set_col(d->ctx->tile_for(d->f64, d->MA));
    hipStream_t st = b.st;
    const int m_old = d->st.basis;
    if (m_old < 1 && !d->eigen) return fail(SSA_ESTATE, "no bidiagonalisation state to continue");
    int fl[4] = {0, 0, 0, 0};
    HIPCHK(hipMemcpy(fl, d->flag, sizeof(fl), hipMemcpyDeviceToHost));
    const bool fresh = fl[2] != 0 || m_old >= d->nshort;
    // per-component buffers for r_new components (the spectrum, the cell
    // sets and the bidiagonalisation state stay)
    for (void* p : {d->T1, d->T2, d->Us, static_cast<void*>(d->U), static_cast<void*>(d->V),
                    static_cast<void*>(d->sigma)})
        d->dfree(p, st);
    d->T1 = d->T2 = d->Us = nullptr;
    d->U = d->V = d->sigma = nullptr;
    const size_t ce = d->celem();
    char *t1, *t2, *us;
    if ((rc = d->dalloc(&t1, d->tslot * ce * r_new)) || (rc = d->dalloc(&t2, d->tslot * ce * r_new)) ||
        (rc = d->dalloc(&us, d->uslot * ce * r_new)) || (rc = d->dalloc(&d->U, d->L * (long)r_new)) ||
        (rc = d->dalloc(&d->V, d->K * (long)r_new)) || (rc = d->dalloc(&d->sigma, r_new))) {
        d->status = rc;
        d->decomposed = false;
        return rc;
    }
    d->T1 = t1; d->T2 = t2; d->Us = us;
    d->op.T1 = d->T1; d->op.T2 = d->T2; d->op.Us = d->Us;
    d->r = r_new;
    d->rs.r = r_new;
    d->rs.U = d->U; d->rs.V = d->V; d->rs.sigma = d->sigma;
    d->lz.r = r_new;
    if ((rc = b.dstep.put(std::vector<int>{0, 0}, st))) return rc;
    d->lz.step = b.dstep.as<int>();
    if ((rc = b.upload_descs())) return rc;
    d->last_st = st;
    const ssa_stats before = d->st;
    auto t0 = Clock::now();
    FinishLists F;
    if (d->eigen && d->Sbig) {
        // the rotated S and its eigenvalues are still resident
        rc = eig_take_big(b, d, r_new);
    } else if (d->eigen) {
        // every eigenpair of S is still resident: take r_new of them
        ItemList I;
        I.h.push_back(Item{0, 0, 0, 0});
        rc = upload_lists({&I}, st);
        if (!rc) launch_eig_take(I.n(), st, b.lzs(), b.res(), I.ptr(), (int)d->L, r_new);
    } else {
        rc = run_lanczos(b, step_limit(), [&] { return finish_lists(b, F); }, m_old, fresh);
    }
    if (!rc) rc = run_finish(b, F);
    d->st.steps += before.steps;
    d->st.restarts += before.restarts + 1;
    d->st.ms_lanczos = before.ms_lanczos + ms_since(t0);
    d->sigma_ready = false;
    d->sigma_h.clear();
    if (rc) {
        d->status = rc;
        d->decomposed = false;
    }
    (void)seal_handle(d);
    return rc ? rc : d->status;
}

namespace {

int check_forecast(ssa_decomp* d, const int* grp, int ng, int h, double* out, int* nseries, const char* what) {
    if (!d) return fail(SSA_EINVAL, "handle is NULL");
    if (!d->rowfam) return fail(SSA_EINVAL, (std::string(what) + " needs a window one row or column wide").c_str());
    if (d->L != (long)d->LB) return fail(SSA_EINVAL, (std::string(what) + " needs a window without mask").c_str());
    if (nseries) *nseries = d->A;
    if (!out) return SSA_OK;
    if (!d->decomposed) return fail(SSA_ESTATE, "not decomposed");
    if (!grp || ng < 1 || h < 1) return fail(SSA_EINVAL, "bad group or horizon");
    if (ng > kVfMaxGroup) return fail(SSA_EINVAL, "forecast group larger than 64 components");
    for (int k = 0; k < ng; ++k)
        if (grp[k] < 0 || grp[k] >= d->r) return fail(SSA_EINVAL, "component id out of range");
    return SSA_OK;
}

// The row forecasts: shift matrix and (I - S^T S)^{-1} of the group's V
// blocks, then the vector (vec = true) or recurrent forecast.
int row_forecast(ssa_decomp* d, const int* grp, int ng, int h, double* out, bool vec) {
    int rc;
    if ((rc = wait_handle(d))) return rc;
    g_tables_ctx = d->ctx;
    TableScope tables(d->ctx, d->ctx->st);
    Batch b(d->ctx);
    b.ds = {d};
    b.f64 = d->f64;
    b.rowfam = d->rowfam;
    b.cls = row_word(d->nh, d->f64);
    b.set_col(d->ctx->tile_for(d->f64, d->MA));
    hipStream_t st = b.st;
    std::vector<int> g(grp, grp + ng);
    const size_t nn = (size_t)ng * ng * sizeof(double);
    DevVec dg, flag, Mr, StS, T, D, G, outd;
    if ((rc = dg.put(g, st)) || (rc = flag.put(std::vector<int>{0, 0}, st)) || (rc = Mr.reserve(nn)) ||
        (rc = StS.reserve(nn)) || (rc = T.reserve(3 * nn)) || (rc = D.reserve(nn)) || (rc = G.reserve(nn)) ||
        (rc = outd.reserve((size_t)d->A * h * sizeof(double))))
        return rc;
    launch_rowf_prep(st, d->kmask, d->KB, d->krow, d->A, d->V, d->K, dg.as<int>(), ng, Mr.as<double>(),
                     StS.as<double>(), T.as<double>(), D.as<double>(), G.as<double>(), flag.as<int>());
    HIPCHK(hipGetLastError());
    DevVec wbuf, rec, yk;
    if (vec) {
        const long E = (long)h + d->KB - 1;   // KB = the longest series' K_p
        if ((rc = wbuf.reserve((size_t)E * ng * sizeof(double)))) return rc;
        ProfSpan p(d->ctx, "vforecast_row", st, [&] { return 8.0 * (2.0 * E * ng + (double)ng * d->K); });
        launch_vrow(st, d->U, d->L, d->sigma, dg.as<int>(), ng, D.as<double>(), E, wbuf.as<double>(), d->V, d->K,
                    d->krow, d->A, h, outd.as<double>());
    } else {
        if ((rc = rec.reserve((size_t)d->A * d->B * sizeof(double))) ||
            (rc = run_reconstruct(b, std::vector<int>{0, ng}, g, {rec.as<double>()})) ||
            (rc = yk.reserve((size_t)h * ng * sizeof(double))))
            return rc;
        ProfSpan p(d->ctx, "rforecast_row", st, [&] { return 8.0 * ((double)ng * d->K + (double)d->A * d->B); });
        launch_rrow(st, d->V, d->K, d->krow, d->A, dg.as<int>(), ng, G.as<double>(), rec.as<double>(), d->B, d->L,
                    h, yk.as<double>(), outd.as<double>());
    }
    HIPCHK(hipGetLastError());
    int bad[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(bad, flag.p, sizeof(bad), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(out, outd.p, (size_t)d->A * h * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (bad[0]) return fail(SSA_EINVAL, "row forecast needs series without gaps");
    if (bad[1]) return fail(SSA_EINVAL, "no row forecast: I - S S^T is singular for the group");
    return SSA_OK;
}

}  // namespace

int ssa_esprit(ssa_decomp* d, const int* grp, int ng, double* re, double* im) {
    CallLock call(d ? d->ctx : nullptr);
    if (!re || !im) return fail(SSA_EINVAL, "NULL argument");
    int rc = check_forecast(d, grp, ng, 1, re, nullptr, "ESPRIT");
    if (rc) return rc;
    if ((rc = wait_handle(d))) return rc;
    g_tables_ctx = d->ctx;
    TableScope tables(d->ctx, d->ctx->st);
    hipStream_t st = d->ctx->st;
    std::vector<int> g(grp, grp + ng);
    DevVec dg, flag, M, dre, dim;
    if ((rc = dg.put(g, st)) || (rc = flag.put(std::vector<int>{0, 0}, st)) ||
        (rc = M.reserve((size_t)ng * ng * sizeof(double))) || (rc = dre.reserve((size_t)ng * sizeof(double))) ||
        (rc = dim.reserve((size_t)ng * sizeof(double))))
        return rc;
    launch_esprit(st, d->U, d->L, dg.as<int>(), ng, M.as<double>(), dre.as<double>(), dim.as<double>(),
                  flag.as<int>());
    HIPCHK(hipGetLastError());
    int bad[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(bad, flag.p, sizeof(bad), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(re, dre.p, (size_t)ng * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(im, dim.p, (size_t)ng * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (bad[0]) return fail(SSA_EINVAL, "no ESPRIT roots: the group's last coordinates have nu^2 >= 1");
    if (bad[1]) return fail(SSA_ENOCONV, "ESPRIT: the eigenvalue iteration did not converge");
    return SSA_OK;
}

int ssa_esprit_noalloc(ssa_decomp* d, const int* grp, int ng, double* re, double* im) {
    CallLock call(d ? d->ctx : nullptr);
    if (!re || !im) return fail(SSA_EINVAL, "NULL argument");
    int rc = check_forecast(d, grp, ng, 1, re, nullptr, "ESPRIT");
    if (rc) return rc;
    // scratch layout: group ids | two flags | shift matrix M | re | im,
    // each region 256-byte aligned
    const auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t og = 0, of = og + up((size_t)ng * sizeof(int)), om = of + up(2 * sizeof(int)),
                 ore = om + up((size_t)ng * ng * sizeof(double)), oim = ore + up((size_t)ng * sizeof(double)),
                 need = oim + up((size_t)ng * sizeof(double));
    if (need > kScratchBytes) return fail(SSA_EINVAL, "group needs more than the 64 KiB fixed scratch");
    unsigned char* base = scratch_of(d->ctx->device);
    if (!base) return fail(SSA_EDEVICE, "device scratch not set up");
    if ((rc = wait_handle(d))) return rc;
    hipStream_t st = d->ctx->st;
    int* dg = reinterpret_cast<int*>(base + og);
    int* flag = reinterpret_cast<int*>(base + of);
    double* M = reinterpret_cast<double*>(base + om);
    double* dre = reinterpret_cast<double*>(base + ore);
    double* dim = reinterpret_cast<double*>(base + oim);
    HIPCHK(hipMemcpyAsync(dg, grp, (size_t)ng * sizeof(int), hipMemcpyHostToDevice, st));
    launch_fill_i32(st, flag, 2, 0);
    launch_esprit(st, d->U, d->L, dg, ng, M, dre, dim, flag);
    HIPCHK(hipGetLastError());
    int bad[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(bad, flag, sizeof(bad), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(re, dre, (size_t)ng * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(im, dim, (size_t)ng * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (bad[0]) return fail(SSA_EINVAL, "no ESPRIT roots: the group's last coordinates have nu^2 >= 1");
    if (bad[1]) return fail(SSA_ENOCONV, "ESPRIT: the eigenvalue iteration did not converge");
    return SSA_OK;
}

int ssa_esprit_tls(ssa_decomp* d, const int* grp, int ng, double* re, double* im) {
    CallLock call(d ? d->ctx : nullptr);
    if (!re || !im) return fail(SSA_EINVAL, "NULL argument");
    int rc = check_forecast(d, grp, ng, 1, re, nullptr, "ESPRIT");
    if (rc) return rc;
    if (ng > kTlsMaxGroup) return fail(SSA_EINVAL, "TLS-ESPRIT group larger than 24 components");
    if ((rc = wait_handle(d))) return rc;
    hipStream_t st = d->ctx->st;
    std::vector<int> g(grp, grp + ng);
    g_tables_ctx = d->ctx;
    DevVec dg, flag, G, dre, dim;
    if ((rc = dg.put(g, st)) || (rc = flag.put(std::vector<int>{0, 0}, st)) ||
        (rc = G.reserve((size_t)4 * ng * ng * sizeof(double))) || (rc = dre.reserve((size_t)ng * sizeof(double))) ||
        (rc = dim.reserve((size_t)ng * sizeof(double))))
        return rc;
    launch_esprit_tls(st, d->U, d->L, dg.as<int>(), ng, G.as<double>(), dre.as<double>(), dim.as<double>(),
                      flag.as<int>());
    HIPCHK(hipGetLastError());
    int bad[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(bad, flag.p, sizeof(bad), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(re, dre.p, (size_t)ng * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(im, dim.p, (size_t)ng * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (bad[0]) return fail(SSA_EINVAL, "no TLS-ESPRIT roots: V22 is singular for the group");
    if (bad[1]) return fail(SSA_ENOCONV, "TLS-ESPRIT: an eigenvalue iteration did not converge");
    return SSA_OK;
}

int ssa_esprit2d(ssa_decomp* d, const int* grp, int ng, double* lre, double* lim, double* mre, double* mim) {
    CallLock call(d ? d->ctx : nullptr);
    if (!d || !grp || !lre || !lim || !mre || !mim) return fail(SSA_EINVAL, "NULL argument");
    if (!d->decomposed) return fail(SSA_ESTATE, "not decomposed");
    if (d->rowfam || d->LA < 2 || d->LB < 2) return fail(SSA_EINVAL, "2D-ESPRIT needs a window at least 2 x 2");
    if (ng < 1 || ng > kVfMaxGroup) return fail(SSA_EINVAL, "group of 1..64 components");
    for (int k = 0; k < ng; ++k)
        if (grp[k] < 0 || grp[k] >= d->r) return fail(SSA_EINVAL, "component id out of range");
    int rc;
    if ((rc = wait_handle(d))) return rc;
    // index pairs in the window's compact order (row-major over its box):
    // per axis the cells whose neighbour one step along it is in the window
    // (with that neighbour), then the cells without such a neighbour
    const int LA = d->LA, LB = d->LB;
    std::vector<int> idx((size_t)LA * LB, -1);
    int c = 0;
    for (int a = 0; a < LA; ++a)
        for (int b = 0; b < LB; ++b)
            if (d->lmask_h[(size_t)a * LB + b]) idx[(size_t)a * LB + b] = c++;
    std::vector<int> lists[4][2];
    for (int ax = 0; ax < 2; ++ax)
        for (int a = 0; a < LA; ++a)
            for (int b = 0; b < LB; ++b) {
                const int i = idx[(size_t)a * LB + b];
                if (i < 0) continue;
                const int a2 = a + (ax == 0), b2 = b + (ax == 1);
                const int j = (a2 < LA && b2 < LB) ? idx[(size_t)a2 * LB + b2] : -1;
                if (j >= 0) {
                    lists[2 * ax][0].push_back(i);
                    lists[2 * ax][1].push_back(j);
                } else {
                    lists[2 * ax + 1][0].push_back(i);
                    lists[2 * ax + 1][1].push_back(i);
                }
            }
    if (lists[0][0].empty() || lists[2][0].empty()) return fail(SSA_EINVAL, "window has no neighbouring cells");
    g_tables_ctx = d->ctx;
    TableScope tables(d->ctx, d->ctx->st);
    hipStream_t st = d->ctx->st;
    std::vector<int> g(grp, grp + ng);
    DevVec dg, flag, dl[4][2], ptrs, gram, T, phi, G, scr, out;
    const size_t nn = (size_t)ng * ng;
    if ((rc = dg.put(g, st)) || (rc = flag.put(std::vector<int>{0, 0, 0}, st))) return rc;
    for (int q = 0; q < 4; ++q)
        for (int h = 0; h < 2; ++h)
            if ((rc = dl[q][h].put(lists[q][h], st))) return rc;
    if ((rc = gram.reserve(2 * nn * sizeof(double))) || (rc = T.reserve(3 * nn * sizeof(double))) ||
        (rc = phi.reserve(2 * nn * sizeof(double))) || (rc = G.reserve(nn * sizeof(double))) ||
        (rc = scr.reserve((3 * nn + 14 * (size_t)ng) * sizeof(double))) ||
        (rc = out.reserve(4 * (size_t)ng * sizeof(double))))
        return rc;
    const int* pa[4] = {dl[0][0].as<int>(), dl[1][0].as<int>(), dl[2][0].as<int>(), dl[3][0].as<int>()};
    const int* pb[4] = {dl[0][1].as<int>(), dl[1][1].as<int>(), dl[2][1].as<int>(), dl[3][1].as<int>()};
    const int np[4] = {(int)lists[0][0].size(), (int)lists[1][0].size(), (int)lists[2][0].size(),
                       (int)lists[3][0].size()};
    launch_esprit2d(st, d->U, d->L, dg.as<int>(), ng, pa, pb, np, gram.as<double>(), T.as<double>(),
                    phi.as<double>(), G.as<double>(), kEsprit2dGamma, scr.as<double>(), out.as<double>(),
                    flag.as<int>());
    HIPCHK(hipGetLastError());
    int bad[3] = {0, 0, 0};
    std::vector<double> h(4 * (size_t)ng);
    HIPCHK(hipMemcpyAsync(bad, flag.p, sizeof(bad), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(h.data(), out.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (bad[1]) return fail(SSA_EINVAL, "2D-ESPRIT: a shift equation is singular for the group");
    if (bad[2]) return fail(SSA_ENOCONV, "2D-ESPRIT: the eigenvalue iteration did not converge");
    for (int k = 0; k < ng; ++k) {
        lre[k] = h[k];
        lim[k] = h[ng + k];
        mre[k] = h[2 * ng + k];
        mim[k] = h[3 * ng + k];
    }
    return SSA_OK;
}

int ssa_rforecast_row(ssa_decomp* d, const int* grp, int ng, int h, double* out, int* nseries) {
    CallLock call(d ? d->ctx : nullptr);
    if (d && d->seg.on)
        return fail(SSA_EINVAL, "forecasts of a series decomposed in segments (longer than one transform row) are not supported");
    int rc = check_forecast(d, grp, ng, h, out, nseries, "row forecast");
    if (rc || !out) return rc;
    return row_forecast(d, grp, ng, h, out, false);
}

int ssa_vforecast_row(ssa_decomp* d, const int* grp, int ng, int h, double* out, int* nseries) {
    CallLock call(d ? d->ctx : nullptr);
    if (d && d->seg.on)
        return fail(SSA_EINVAL, "forecasts of a series decomposed in segments (longer than one transform row) are not supported");
    int rc = check_forecast(d, grp, ng, h, out, nseries, "row forecast");
    if (rc || !out) return rc;
    return row_forecast(d, grp, ng, h, out, true);
}

int ssa_reconstruct_batch_dev(int n, ssa_decomp* const* d, const int* gp, const int* gi, int ng,
                              double* const* out_dev) {
    CallLock call(n > 0 && d && d[0] ? d[0]->ctx : nullptr);
    if (n <= 0 || !d || !out_dev) return fail(SSA_EINVAL, "bad arguments");
    for (int i = 0; i < n; ++i)
        if (d[i] && d[i]->seg.on)
            return fail(SSA_EINVAL, "device reconstruction of a series decomposed in segments is not supported");
    for (int i = 0; i < n; ++i) {
        if (!d[i] || !d[i]->decomposed) return fail(SSA_ESTATE, "not decomposed");
        if (geo_key(d[i]) != geo_key(d[0])) return fail(SSA_EINVAL, "handles differ in kernel class");
        if (d[i]->tr) return fail(SSA_EINVAL, "device reconstruction needs a window more than one column wide");
    }
    int rc = SSA_OK;
    for (int i = 0; i < n && !rc; ++i) rc = check_groups(d[i], gp, gi, ng);
    if (rc) return rc;
    g_tables_ctx = d[0]->ctx;
    TableScope tables(d[0]->ctx, d[0]->ctx->st);
    Batch b(d[0]->ctx);
    b.ds.assign(d, d + n);
    b.f64 = d[0]->f64;
    b.rowfam = d[0]->rowfam;
    b.cls = row_word(d[0]->nh, d[0]->f64);
    b.set_col(d[0]->ctx->tile_for(d[0]->f64, d[0]->MA));
    return run_reconstruct(b, std::vector<int>(gp, gp + ng + 1), std::vector<int>(gi, gi + gp[ng]),
                           std::vector<double*>(out_dev, out_dev + n));
}

int ssa_get_stats(const ssa_decomp* d, ssa_stats* st) {
    if (!d || !st) return fail(SSA_EINVAL, "NULL argument");
    *st = d->st;
    st->device_bytes = d->bytes;
    st->fft_rows = d->rowfam ? d->A : d->MA;
    st->fft_cols = d->MB;
    return SSA_OK;
}

void ssa_free(ssa_decomp* d) { delete d; }

int ssa_submit(ssa_ctx* ctx, const ssa_request* req, const int* grp_ptr, const int* grp_idx, int ngroups,
               uint64_t* ticket) {
    if (!ctx || !req || !ticket) return fail(SSA_EINVAL, "NULL argument");
    // The worker threads run only with SHSSA_SERVE_ENGINE set (a GPU fault
    // seen once on them is not explained); by default the server is
    // cooperative: ssa_poll and ssa_wait drive the requests.
    const bool engine = std::getenv("SHSSA_SERVE_ENGINE") != nullptr;
    if (!req->x || req->nx <= 0 || req->ny <= 0) return fail(SSA_EINVAL, "sizes must be positive");
    if (ngroups < 0 || (ngroups > 0 && (!grp_ptr || !grp_idx))) return fail(SSA_EINVAL, "bad groups");
    auto r = std::make_shared<ServeReq>();
    const size_t n = (size_t)req->nx * req->ny;
    r->x.assign(req->x, req->x + n);
    r->q = *req;
    r->q.x = r->x.data();
    if (req->mask) {
        r->mask.assign(req->mask, req->mask + n);
        r->q.mask = r->mask.data();
    }
    if (req->wmask) {
        r->wmask.assign(req->wmask, req->wmask + (size_t)req->lx * req->ly);
        r->q.wmask = r->wmask.data();
    }
    if (ngroups > 0) {
        r->gp.assign(grp_ptr, grp_ptr + ngroups + 1);
        r->gi.assign(grp_idx, grp_idx + grp_ptr[ngroups]);
    }
    r->d.reset(new ssa_decomp());
    int rc = plan_request(ctx, r->q, r->d.get());
    if (rc) return rc;
    if (ngroups > 0 && (rc = check_groups(r->d.get(), r->gp.data(), r->gi.data(), ngroups))) return rc;
    r->key = geo_key(r->d.get());
    r->est = estimate_bytes(r->d.get(), ngroups);
    if (ctx->budget && r->est > ctx->budget)
        return fail(SSA_ENOMEM, "request larger than the context's memory budget");
    if ((rc = engine ? serve_start(ctx) : coop_start(ctx))) return rc;
    Server& S = *ctx->srv;
    if (engine == (S.coop != nullptr))
        return fail(SSA_ESTATE, "SHSSA_SERVE_ENGINE changed after the context's first request");
    {
        std::lock_guard<std::mutex> lk(S.mu);
        r->ticket = S.next++;
        r->t_submit = S.now();
        S.reqs[r->ticket] = r;
        S.pending.push_back(r);
        *ticket = r->ticket;
    }
    S.cv.notify_all();
    return SSA_OK;
}

int ssa_submit_multi(ssa_ctx* ctx, const double* const* series, const int* len, int s, int L, int r,
                     int precision, const int* grp_ptr, const int* grp_idx, int ngroups, uint64_t* ticket) {
    if (!series || !len || s <= 0) return fail(SSA_EINVAL, "no series");
    int nmax = 0, nmin = 1 << 30;
    for (int p = 0; p < s; ++p) {
        if (len[p] <= 0 || !series[p]) return fail(SSA_EINVAL, "empty series");
        nmax = std::max(nmax, len[p]);
        nmin = std::min(nmin, len[p]);
    }
    if (!(L > 1 && L < nmin)) return fail(SSA_EINVAL, "window must satisfy 1 < L < min N_p");
    std::vector<double> x((size_t)nmax * s, std::nan(""));
    for (int p = 0; p < s; ++p)
        for (int t = 0; t < len[p]; ++t) x[(size_t)t * s + p] = series[p][t];
    ssa_request q{x.data(), nmax, s, nullptr, nullptr, L, 1, r, precision, 0x5eedULL};
    return ssa_submit(ctx, &q, grp_ptr, grp_idx, ngroups, ticket);
}

int ssa_poll(ssa_ctx* ctx, uint64_t ticket, int* done) {
    if (!ctx || !done) return fail(SSA_EINVAL, "NULL argument");
    if (!ctx->srv) return fail(SSA_EINVAL, "unknown ticket");
    Server& S = *ctx->srv;
    bool d = false;
    if (!find_ticket(S, ticket, &d)) return fail(SSA_EINVAL, "unknown ticket");
    if (!d && S.coop) {
        // cooperative server: one round of work
        CallLock call(ctx);
        if (int rc = coop_advance(ctx)) return rc;
        (void)find_ticket(S, ticket, &d);
    }
    *done = d;
    return SSA_OK;
}

int ssa_wait(ssa_ctx* ctx, uint64_t ticket) {
    if (!ctx || !ctx->srv) return fail(SSA_EINVAL, "unknown ticket");
    Server& S = *ctx->srv;
    if (S.coop) {
        for (;;) {
            bool d = false;
            if (!find_ticket(S, ticket, &d)) return fail(SSA_EINVAL, "unknown ticket");
            if (d) return SSA_OK;
            CallLock call(ctx);
            if (int rc = coop_advance(ctx)) return rc;
        }
    }
    std::unique_lock<std::mutex> lk(S.mu);
    auto it = S.reqs.find(ticket);
    if (it == S.reqs.end()) return fail(SSA_EINVAL, "unknown ticket");
    auto r = it->second;
    S.cv.wait(lk, [&] { return r->done; });
    return SSA_OK;
}

int ssa_take(ssa_ctx* ctx, uint64_t ticket, ssa_decomp** out, double* recon, ssa_times* times) {
    if (!ctx || !out) return fail(SSA_EINVAL, "NULL argument");
    *out = nullptr;
    if (!ctx->srv) return fail(SSA_EINVAL, "unknown ticket");
    Server& S = *ctx->srv;
    std::shared_ptr<ServeReq> r;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        auto it = S.reqs.find(ticket);
        if (it == S.reqs.end()) return fail(SSA_EINVAL, "unknown ticket");
        if (!it->second->done) return SSA_EBUSY;
        r = it->second;
        S.reqs.erase(it);
    }
    if (times) {
        times->queue_ms = r->t_start - r->t_submit;
        times->total_ms = r->t_done - r->t_submit;
    }
    const int st = r->status;
    if (st == SSA_OK || st == SSA_ENOCONV) {
        if (recon && !r->recon.empty()) std::memcpy(recon, r->recon.data(), r->recon.size() * sizeof(double));
        *out = r->d.release();
    }
    return st == SSA_OK ? SSA_OK : fail(st, "request failed");
}

const char* ssa_strerror(int code) {
    switch (code) {
    case SSA_OK: return "ok";
    case SSA_EINVAL: return "invalid argument";
    case SSA_EEMPTY: return "no window position fits inside the array";
    case SSA_ERANK: return "r must satisfy 1 <= r < min(L, K)";
    case SSA_ENOMEM: return "out of device memory";
    case SSA_ENOCONV: return "bidiagonalisation did not converge";
    case SSA_EDEVICE: return "HIP runtime error";
    case SSA_EBUSY: return "request not finished";
    case SSA_ESTATE: return "call out of order";
    default: return "unknown error";
    }
}

const char* ssa_last_error(void) { return g_err.c_str(); }

}  // extern "C"
