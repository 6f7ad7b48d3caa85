// Host-only stand-in for the HIP runtime, for auditing the library's host
// code (scheduler, pool, deferred frees, staging) under AddressSanitizer or
// ThreadSanitizer on a machine without a GPU.
//
// Device memory is host heap memory.  Each stream is a thread that runs its
// queue in order (copies, kernel launches, event records), slowly enough for
// work to pile up, so the ordering between host decisions and queued work is
// the asynchronous one of a real device.  Kernels do not compute: when one
// runs, the mock reads one byte at every pointer argument and at every
// pointer field of the descriptors its work items name (the sanitizer then
// reports a launch that refers to freed memory), and it fills in the few
// outputs that steer the host (origin counts, row offsets, convergence
// flags).  The library's pool calls shssa_audit_block() (built with
// SHSSA_HOST_AUDIT) whenever a block becomes free for reuse; the mock
// reports the block if queued, unfinished work still refers to it.
//
// Environment: MOCK_OP_US (microseconds per queued operation, default 30),
// MOCK_DEVICE_BYTES (hipMalloc fails beyond this many live bytes).
#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <cxxabi.h>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../paper_1309_5050_amd/csrc/device.hpp"

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#include <sanitizer/asan_interface.h>
#define MOCK_POISON(p, n) ASAN_POISON_MEMORY_REGION(p, n)
#define MOCK_UNPOISON(p, n) ASAN_UNPOISON_MEMORY_REGION(p, n)
#endif
#endif
#ifndef MOCK_POISON
#define MOCK_POISON(p, n) ((void)(p), (void)(n))
#define MOCK_UNPOISON(p, n) ((void)(p), (void)(n))
#endif

using shssa::Item;
using shssa::LzDesc;
using shssa::OpDesc;
using shssa::ResDesc;

namespace {

std::atomic<int> g_errors{0};

void report(const char* what) {
    g_errors++;
    std::fprintf(stderr, "MOCK-AUDIT: %s\n", what);
}

// ---- allocations (also filled by static constructors: built on first use)
std::mutex& amu() {
    static std::mutex m;
    return m;
}
std::map<uintptr_t, size_t>& live_map() {   // device blocks and device variables: base -> bytes
    static std::map<uintptr_t, size_t> m;
    return m;
}
size_t g_live_bytes = 0;

size_t device_cap() {
    static size_t cap = [] {
        const char* e = std::getenv("MOCK_DEVICE_BYTES");
        return e ? (size_t)std::strtoull(e, nullptr, 10) : (size_t)0;
    }();
    return cap;
}

bool trace() {
    static bool t = std::getenv("MOCK_TRACE") != nullptr;
    return t;
}

int op_us() {
    static int us = [] {
        const char* e = std::getenv("MOCK_OP_US");
        return e ? std::atoi(e) : 30;
    }();
    return us;
}

inline void touch(const void* p) {
    if (!p) return;
    const volatile unsigned char* c = static_cast<const volatile unsigned char*>(p);
    (void)*c;
}

// p inside a live device block
bool live(const void* p) {
    const auto a = reinterpret_cast<uintptr_t>(p);
    std::lock_guard<std::mutex> g(amu());
    auto it = live_map().upper_bound(a);
    if (it == live_map().begin()) return false;
    --it;
    return a < it->first + std::max<size_t>(it->second, 1);
}

thread_local const char* t_kernel = "";

// a descriptor field of a running kernel: reported (and not read) when it
// points outside every live device block
inline void field(const void* p, const char* what) {
    if (!p) return;
    if (!live(p)) {
        char buf[200];
        std::snprintf(buf, sizeof buf, "%s: %s = %p is not in a live device block", t_kernel, what, p);
        report(buf);
        return;
    }
    touch(p);
}

// ---- kernels registered by the library's objects (registration runs in
// the objects' static constructors, so the table is built on first use)
std::mutex& kmu() {
    static std::mutex m;
    return m;
}
std::map<const void*, std::string>& kernels() {   // host stub -> demangled signature
    static std::map<const void*, std::string> k;
    return k;
}

struct KernelInfo {
    std::string name;                 // without parameters
    std::vector<std::string> params;  // parameter types
};

KernelInfo parse(const std::string& sig) {
    KernelInfo k;
    const size_t lp = sig.find('(');
    k.name = sig.substr(0, lp);
    if (k.name.rfind("void ", 0) == 0) k.name = k.name.substr(5);
    const size_t tl = k.name.find('<');
    if (tl != std::string::npos) k.name = k.name.substr(0, tl);
    if (lp == std::string::npos) return k;
    int depth = 0;
    std::string cur;
    for (size_t i = lp + 1; i < sig.size(); ++i) {
        const char c = sig[i];
        if (c == '<' || c == '(') depth++;
        if (c == '>' || c == ')') {
            if (depth == 0) break;
            depth--;
        }
        if (c == ',' && depth == 0) {
            k.params.push_back(cur);
            cur.clear();
            continue;
        }
        if (!(cur.empty() && c == ' ')) cur += c;
    }
    if (!cur.empty()) k.params.push_back(cur);
    return k;
}

// ---- streams and events
struct Op {
    std::function<void()> run;
    std::vector<std::pair<const void*, size_t>> refs;   // memory the operation uses
};

struct MockStream {
    std::mutex m;
    std::condition_variable cv;
    std::deque<Op> q;
    uint64_t enq = 0, done = 0;
    bool stop = false;
    std::thread th;
    void loop() {
        for (;;) {
            Op op;
            {
                std::unique_lock<std::mutex> lk(m);
                cv.wait(lk, [&] { return stop || !q.empty(); });
                if (q.empty()) return;
                op = q.front();
            }
            if (op_us() > 0) std::this_thread::sleep_for(std::chrono::microseconds(op_us()));
            op.run();
            {
                std::lock_guard<std::mutex> lk(m);
                q.pop_front();
                done++;
            }
            cv.notify_all();
        }
    }
    void push(Op op) {
        {
            std::lock_guard<std::mutex> lk(m);
            q.push_back(std::move(op));
            enq++;
        }
        cv.notify_all();
    }
    void drain() {
        std::unique_lock<std::mutex> lk(m);
        cv.wait(lk, [&] { return q.empty(); });
    }
};

std::mutex g_smu;
std::vector<MockStream*> g_streams;

MockStream* null_stream() {
    static MockStream* s = [] {
        auto* x = new MockStream();
        x->th = std::thread([x] { x->loop(); });
        std::lock_guard<std::mutex> g(g_smu);
        g_streams.push_back(x);
        return x;
    }();
    return s;
}

MockStream* S(hipStream_t s) { return s ? reinterpret_cast<MockStream*>(s) : null_stream(); }

// An event refers to its stream until the stream is destroyed (its work has
// then completed, so the event has too).
struct MockEvent {
    MockStream* s = nullptr;
    uint64_t ticket = 0;
};
std::mutex g_emu;   // guards every event's stream pointer; taken before a stream's lock
std::map<MockEvent*, int> g_events;

bool event_complete(MockEvent* e) {
    std::lock_guard<std::mutex> g(g_emu);
    if (!e->s) return true;
    std::lock_guard<std::mutex> lk(e->s->m);
    return e->s->done >= e->ticket;
}

// pending (queued, unfinished) operations of every stream that use [p, p + n)
int pending_refs(const void* p, size_t n, MockStream* except) {
    const auto lo = reinterpret_cast<uintptr_t>(p), hi = lo + n;
    int hits = 0;
    std::lock_guard<std::mutex> g(g_smu);
    for (MockStream* s : g_streams) {
        if (s == except) continue;
        std::lock_guard<std::mutex> lk(s->m);
        for (const Op& op : s->q)
            for (const auto& r : op.refs) {
                const auto a = reinterpret_cast<uintptr_t>(r.first);
                if (a < hi && a + std::max<size_t>(r.second, 1) > lo) hits++;
            }
    }
    return hits;
}

// ---- kernel execution: touches and the outputs that steer the host
struct Launch {
    KernelInfo k;
    dim3 grid, block;
    std::vector<const void*> ptrs;    // pointer arguments (nullptr for non-pointers)
    std::vector<long long> ints;      // integer arguments (0 for others)
    bool step = false;                // the kernel reads the instances' step counters
};

// the step counter only where the launch reads it (handles keep no counter
// between batches)
void touch_lz(const LzDesc& z, bool step) {
    if (step && !z.step) report((std::string(t_kernel) + ": reads a null LzDesc.step").c_str());
    if (step) field(z.step, "LzDesc.step"); field(z.Q, "LzDesc.Q"); field(z.Q32, "LzDesc.Q32"); field(z.w, "LzDesc.w");
    field(z.sin, "LzDesc.sin"); field(z.hp1, "LzDesc.hp1"); field(z.hp2, "LzDesc.hp2"); field(z.np, "LzDesc.np");
    field(z.np0, "LzDesc.np0"); field(z.lbuf[0], "LzDesc.lbuf0"); field(z.lbuf[1], "LzDesc.lbuf1");
    field(z.lnp[0], "LzDesc.lnp0"); field(z.lnp[1], "LzDesc.lnp1"); field(z.gam, "LzDesc.gam");
    field(z.Bm, "LzDesc.Bm"); field(z.Yl, "LzDesc.Yl"); field(z.Yr, "LzDesc.Yr"); field(z.sig, "LzDesc.sig");
    field(z.perm, "LzDesc.perm"); field(z.beta, "LzDesc.beta"); field(z.flag, "LzDesc.flag");
    field(z.Qtmp, "LzDesc.Qtmp");
}
void touch_op(const OpDesc& o) {
    for (int s = 0; s < 2; ++s) {
        field(o.S[s].mask, "OpDesc.S.mask"); field(o.S[s].rowoff, "OpDesc.S.rowoff");
        field(o.S[s].pref, "OpDesc.S.pref");
    }
    field(o.prow.tw, "OpDesc.prow.tw"); field(o.prow.twr, "OpDesc.prow.twr"); field(o.pcol.tw, "OpDesc.pcol.tw");
    field(o.pcol.twr, "OpDesc.pcol.twr"); field(o.Xh, "OpDesc.Xh"); field(o.T1, "OpDesc.T1");
    field(o.T2, "OpDesc.T2"); field(o.Us, "OpDesc.Us"); field(o.W, "OpDesc.W"); field(o.xc, "OpDesc.xc");
    field(o.nset, "OpDesc.nset");
}
void touch_res(const ResDesc& r) {
    field(r.U, "ResDesc.U"); field(r.V, "ResDesc.V"); field(r.sigma, "ResDesc.sigma");
    field(r.recon, "ResDesc.recon"); field(r.gptr, "ResDesc.gptr"); field(r.gidx, "ResDesc.gidx");
}

void run_kernel(const Launch& L) {
    const auto& P = L.k.params;
    t_kernel = L.k.name.c_str();
    for (size_t i = 0; i < L.ptrs.size(); ++i) field(L.ptrs[i], P[i].c_str());
    // descriptors of the instances the work items name
    int items_at = -1;
    for (size_t i = 0; i < P.size(); ++i)
        if (P[i] == "shssa::Item const*" && L.ptrs[i]) items_at = (int)i;
    if (items_at >= 0) {
        const Item* it = static_cast<const Item*>(L.ptrs[items_at]);
        for (unsigned b = 0; b < L.grid.x; ++b) {
            const int inst = it[b].inst;
            for (size_t i = 0; i < P.size(); ++i) {
                if (!L.ptrs[i]) continue;
                if (P[i] == "shssa::LzDesc const*") touch_lz(static_cast<const LzDesc*>(L.ptrs[i])[inst], L.step);
                if (P[i] == "shssa::OpDesc const*") touch_op(static_cast<const OpDesc*>(L.ptrs[i])[inst]);
                if (P[i] == "shssa::ResDesc const*") touch_res(static_cast<const ResDesc*>(L.ptrs[i])[inst]);
            }
        }
    }
    const std::string& n = L.k.name;
    if (n == "shssa::k_shape_origins") {
        // every origin of a full window inside an unmasked array counts
        const auto* ops = static_cast<const OpDesc*>(L.ptrs[0]);
        const auto* it = static_cast<const Item*>(L.ptrs[1]);
        auto* const* kmask = static_cast<uint8_t* const*>(L.ptrs[4]);
        int* const* kcount = static_cast<int* const*>(L.ptrs[6]);
        for (unsigned b = 0; b < L.grid.x; ++b) {
            const OpDesc& o = ops[it[b].inst];
            const int KB = o.S[1].boxB;
            std::memset(kmask[it[b].inst] + (long)it[b].idx * KB, 1, (size_t)KB);
            kcount[it[b].inst][it[b].idx] = KB;
        }
    } else if (n == "shssa::k_shape_rowoff") {
        const int ninst = (int)L.ints[0];
        const int* const* kcount = static_cast<const int* const*>(L.ptrs[1]);
        int* const* rowoff = static_cast<int* const*>(L.ptrs[2]);
        const int* nrows = static_cast<const int*>(L.ptrs[3]);
        long* total = static_cast<long*>(const_cast<void*>(L.ptrs[4]));
        for (int i = 0; i < ninst && i < (int)L.grid.x; ++i) {
            long s = 0;
            for (int a = 0; a < nrows[i]; ++a) {
                rowoff[i][a] = (int)s;
                s += kcount[i][a];
            }
            rowoff[i][nrows[i]] = (int)s;
            total[i] = s;
        }
    } else if (n == "shssa::k_lz_svd") {
        const auto* lzs = static_cast<const LzDesc*>(L.ptrs[0]);
        const auto* it = static_cast<const Item*>(L.ptrs[1]);
        const int m = (int)L.ints[2];
        for (unsigned b = 0; b < L.grid.x; ++b) {
            const LzDesc& z = lzs[it[b].inst];
            z.flag[0] = 1;   // converged
            z.flag[1] = 1;
            z.beta[1] = 0.0;
            for (int i = 0; i < m; ++i) {
                z.perm[i] = i;
                z.sig[i] = 1.0;
            }
        }
    } else if (n == "shssa::k_gather_flags") {
        const auto* lzs = static_cast<const LzDesc*>(L.ptrs[0]);
        const int ninst = (int)L.ints[1];
        int* flags = static_cast<int*>(const_cast<void*>(L.ptrs[2]));
        double* betas = static_cast<double*>(const_cast<void*>(L.ptrs[3]));
        for (int i = 0; i < ninst; ++i) {
            for (int k = 0; k < 4; ++k) flags[4 * i + k] = lzs[i].flag[k];
            for (int k = 0; k < 2; ++k) betas[2 * i + k] = lzs[i].beta[k];
        }
    }
}

thread_local dim3 t_grid, t_block;
thread_local size_t t_shm = 0;
thread_local hipStream_t t_st = nullptr;

}  // namespace

extern "C" {

// audit hooks of the library's pool.  A block entering the pool (reuse_on
// null) or reused at once on stream reuse_on must have no queued user left
// (on other streams than reuse_on); a pooled block is poisoned for the
// address sanitizer until it leaves the pool, so queued work that reaches it
// through a descriptor is reported where it reads.
void shssa_audit_block(const void* p, size_t n, hipStream_t reuse_on) {
    MockStream* except = reuse_on ? S(reuse_on) : nullptr;
    const int h = pending_refs(p, n, except);
    if (h) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "block %p (%zu bytes) freed for reuse while %d queued operations use it", p,
                      n, h);
        report(buf);
    }
    if (!reuse_on) MOCK_POISON(p, n);
}
void shssa_audit_take(const void* p, size_t n) { MOCK_UNPOISON(p, n); }

int mock_audit_errors() { return g_errors.load(); }

// ---- registration
void** __hipRegisterFatBinary(const void*) {
    static void* handle = nullptr;
    return &handle;
}
void __hipUnregisterFatBinary(void**) {}
void __hipRegisterFunction(void**, const void* hostFunction, char*, const char* deviceName, unsigned int, void*,
                           void*, void*, void*, int*) {
    int st = 0;
    char* dm = abi::__cxa_demangle(deviceName, nullptr, nullptr, &st);
    std::lock_guard<std::mutex> g(kmu());
    kernels()[hostFunction] = dm ? std::string(dm) : std::string(deviceName);
    std::free(dm);
}
void __hipRegisterVar(void**, void* var, char*, char*, int, size_t size, int, int) {
    std::lock_guard<std::mutex> g(amu());
    live_map()[reinterpret_cast<uintptr_t>(var)] = size;
}

hipError_t __hipPushCallConfiguration(dim3 g, dim3 b, size_t shm, hipStream_t st) {
    t_grid = g;
    t_block = b;
    t_shm = shm;
    t_st = st;
    return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3* g, dim3* b, size_t* shm, hipStream_t* st) {
    *g = t_grid;
    *b = t_block;
    *shm = t_shm;
    *st = t_st;
    return hipSuccess;
}

hipError_t hipLaunchKernel(const void* f, dim3 grid, dim3 block, void** args, size_t, hipStream_t st) {
    Launch L;
    {
        std::lock_guard<std::mutex> g(kmu());
        auto it = kernels().find(f);
        if (it == kernels().end()) {
            report("launch of an unregistered kernel");
            return hipErrorInvalidDeviceFunction;
        }
        L.k = parse(it->second);
    }
    L.grid = grid;
    L.block = block;
    if (grid.x == 0 || block.x == 0 || block.x * block.y * block.z > 1024) {
        report(("launch shape out of range: " + L.k.name).c_str());
        return hipErrorInvalidConfiguration;
    }
    Op op;
    for (size_t i = 0; i < L.k.params.size(); ++i) {
        const std::string& t = L.k.params[i];
        const void* p = nullptr;
        long long v = 0;
        if (!t.empty() && t.back() == '*') {
            p = *static_cast<const void* const*>(args[i]);
            if (p) op.refs.push_back({p, 1});
        } else if (t == "int") {
            v = *static_cast<const int*>(args[i]);
        } else if (t == "long" || t == "unsigned long long") {
            v = *static_cast<const long long*>(args[i]);
        } else if (t == "shssa::RowInArgs") {
            L.step |= static_cast<const shssa::RowInArgs*>(args[i])->mode == shssa::IN_LZ_STEP;
        } else if (t == "shssa::RowMidArgs") {
            L.step |= static_cast<const shssa::RowMidArgs*>(args[i])->j == shssa::kStepDev;
        } else if (t == "shssa::RowOutArgs") {
            L.step |= static_cast<const shssa::RowOutArgs*>(args[i])->j == shssa::kStepDev;
        } else if (t == "shssa::RowFamArgs") {
            L.step |= static_cast<const shssa::RowFamArgs*>(args[i])->j == shssa::kStepDev;
        }
        L.ptrs.push_back(p);
        L.ints.push_back(v);
    }
    const std::string& kn = L.k.name;
    if (kn == "shssa::k_step_set" || kn == "shssa::k_step_next_inst") L.step = true;
    if ((kn == "shssa::k_lz_proj" || kn == "shssa::k_lz_proj2" || kn == "shssa::k_lz_update") && L.ints.size() > 2 &&
        L.ints[2] < 0)
        L.step = true;   // column count from the step counter
    if (trace()) std::fprintf(stderr, "launch %s grid %u stream %p\n", L.k.name.c_str(), grid.x, (void*)st);
    op.run = [L] { run_kernel(L); };
    S(st)->push(std::move(op));
    return hipSuccess;
}

// ---- device
hipError_t hipGetDeviceCount(int* n) {
    *n = 1;
    return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "mock runtime error"; }
hipError_t hipDeviceSynchronize() {
    std::vector<MockStream*> ss;
    {
        std::lock_guard<std::mutex> g(g_smu);
        ss = g_streams;
    }
    for (auto* s : ss) s->drain();
    return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** p, const void* sym) {
    *p = const_cast<void*>(sym);
    return hipSuccess;
}

// ---- memory
hipError_t hipMalloc(void** p, size_t n) {
    std::lock_guard<std::mutex> g(amu());
    if (device_cap() && g_live_bytes + n > device_cap()) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    *p = std::calloc(1, std::max<size_t>(n, 1));
    live_map()[reinterpret_cast<uintptr_t>(*p)] = n;
    g_live_bytes += n;
    return hipSuccess;
}
hipError_t hipFree(void* p) {
    if (!p) return hipSuccess;
    if (const int h = pending_refs(p, 1, nullptr)) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "hipFree(%p) while %d queued operations use it", p, h);
        report(buf);
    }
    {
        std::lock_guard<std::mutex> g(amu());
        auto it = live_map().find(reinterpret_cast<uintptr_t>(p));
        if (it == live_map().end()) {
            report("hipFree of a pointer that hipMalloc did not return (or freed twice)");
            return hipErrorInvalidValue;
        }
        g_live_bytes -= it->second;
        live_map().erase(it);
    }
    std::free(p);
    return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned int) {
    *p = std::calloc(1, std::max<size_t>(n, 1));
    return hipSuccess;
}
hipError_t hipHostFree(void* p) {
    if (const int h = pending_refs(p, 1, nullptr)) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "hipHostFree(%p) while %d queued copies use it", p, h);
        report(buf);
    }
    std::free(p);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t st) {
    Op op;
    op.refs = {{dst, n}, {src, n}};
    op.run = [dst, src, n] {
        if (n) std::memcpy(dst, src, n);
    };
    S(st)->push(std::move(op));
    return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind) {
    // the null stream: runs in order behind the null stream's earlier work
    hipMemcpyAsync(dst, src, n, hipMemcpyDefault, nullptr);
    null_stream()->drain();
    return hipSuccess;
}

// ---- streams
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
    auto* x = new MockStream();
    x->th = std::thread([x] { x->loop(); });
    {
        std::lock_guard<std::mutex> g(g_smu);
        g_streams.push_back(x);
    }
    *s = reinterpret_cast<hipStream_t>(x);
    return hipSuccess;
}
hipError_t hipStreamCreate(hipStream_t* s) { return hipStreamCreateWithFlags(s, 0); }
hipError_t hipStreamSynchronize(hipStream_t s) {
    if (trace()) std::fprintf(stderr, "sync stream %p\n", (void*)s);
    S(s)->drain();
    if (trace()) std::fprintf(stderr, "synced stream %p\n", (void*)s);
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    MockStream* x = S(s);
    x->drain();
    {
        std::lock_guard<std::mutex> lk(x->m);
        x->stop = true;
    }
    x->cv.notify_all();
    x->th.join();
    {
        std::lock_guard<std::mutex> g(g_emu);
        for (auto& kv : g_events)
            if (kv.first->s == x) kv.first->s = nullptr;
    }
    {
        std::lock_guard<std::mutex> g(g_smu);
        for (size_t i = 0; i < g_streams.size(); ++i)
            if (g_streams[i] == x) {
                g_streams.erase(g_streams.begin() + (long)i);
                break;
            }
    }
    delete x;
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipErrorNotSupported; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t*) { return hipErrorNotSupported; }
hipError_t hipGraphInstantiate(hipGraphExec_t*, hipGraph_t, hipGraphNode_t*, char*, size_t) {
    return hipErrorNotSupported;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }

// ---- events
hipError_t hipEventCreate(hipEvent_t* e) {
    auto* ev = new MockEvent();
    {
        std::lock_guard<std::mutex> g(g_emu);
        g_events[ev] = 1;
    }
    *e = reinterpret_cast<hipEvent_t>(ev);
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
    auto* ev = reinterpret_cast<MockEvent*>(e);
    {
        std::lock_guard<std::mutex> g(g_emu);
        g_events.erase(ev);
    }
    delete ev;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    auto* ev = reinterpret_cast<MockEvent*>(e);
    MockStream* x = S(s);
    std::lock_guard<std::mutex> g(g_emu);
    std::lock_guard<std::mutex> lk(x->m);
    ev->s = x;
    ev->ticket = x->enq;
    return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
    return event_complete(reinterpret_cast<MockEvent*>(e)) ? hipSuccess : hipErrorNotReady;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
    auto* ev = reinterpret_cast<MockEvent*>(e);
    if (trace()) std::fprintf(stderr, "event sync %p\n", (void*)e);
    while (!event_complete(ev)) std::this_thread::sleep_for(std::chrono::microseconds(50));
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
    *ms = 0.01f;
    return hipSuccess;
}

}  // extern "C"
