// Host-only stand-in for the HIP runtime.  It is linked into a host-only
// build of the library (kernels compiled out) so that the library's host
// code can run on a machine without a GPU under AddressSanitizer and
// UndefinedBehaviorSanitizer.  It models what decides whether host code is
// correct, not what the kernels compute:
//
//  * device memory: every hipMalloc is an anonymous mapping with no access
//    rights, so a host dereference of a device pointer faults at the
//    instruction that makes it; the stub opens exactly the pages a copy or a
//    fill touches and closes them again.  Freed allocations stay reserved
//    and are never reused, so a later use of one is reported as such;
//  * asynchronous work: copies enqueued on a stream run only when a call
//    that completes that stream runs (stream, event or device
//    synchronisation, a blocking copy, hipFree, hipHostFree, stream
//    destruction).  A host buffer freed or out of scope before that point is
//    reported, with the place the copy was enqueued;
//  * graph capture: work enqueued while a stream captures is recorded (and
//    follows event waits into other streams); every hipGraphLaunch enqueues
//    the recorded copies again, and they read the host memory they name when
//    they run.  A blocking call, an allocation or a fill during capture is
//    an error;
//  * kernels do not run; the launch shape and the dynamic LDS size are
//    checked against gfx950's limits and the kernel must be registered.
//
// Any breach prints a line starting with "HOSTCHECK:" and the stack, then
// aborts.  Device memory reads back as zeros unless a copy wrote it.
//
// Error paths: with HOSTCHECK_FAIL_AT=k in the environment the k-th fallible
// call (allocation, copy, launch, stream/event/graph creation, capture,
// synchronisation) fails with the error the runtime would return; with
// HOSTCHECK_FAIL_SITE=k the first call made from the k-th distinct call
// site (its callers' return addresses) fails.  Either runs one of the
// library's error returns under the sanitizers.
#include <hip/hip_runtime_api.h>
#include <sanitizer/asan_interface.h>
#include <sanitizer/common_interface_defs.h>
#include <sys/mman.h>
#include <unistd.h>

#include <algorithm>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <execinfo.h>
#include <map>
#include <mutex>
#include <set>
#include <vector>

struct ihipGraph;

namespace {

constexpr size_t kPage = 4096;
constexpr size_t kLdsMax = 160 * 1024;                       // LDS per workgroup
constexpr size_t kHbm = 288ull << 30;                        // HBM3E per GPU
constexpr int kCus = 256;

struct Site {
    void* pc[20];
    int n = 0;
    void capture() { n = backtrace(pc, 20); }
    void print(const char* what) const {
        fprintf(stderr, "HOSTCHECK: %s\n", what);
        for (int i = 2; i < n; ++i) {   // skip the stub's own frames
            char buf[512];
            __sanitizer_symbolize_pc(pc[i], "%p %F %L", buf, sizeof buf);
            fprintf(stderr, "    #%d %s\n", i - 2, buf);
        }
    }
};

[[noreturn]] void fail(const Site* site, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    fprintf(stderr, "HOSTCHECK: ");
    vfprintf(stderr, fmt, ap);
    fputc('\n', stderr);
    va_end(ap);
    if (site) site->print("the work was enqueued at:");
    fprintf(stderr, "HOSTCHECK: reported from:\n");
    __sanitizer_print_stack_trace();
    fflush(stderr);
    abort();
}

enum OpKind { OP_COPY, OP_COPY2D, OP_KERNEL, OP_WAIT };

}  // namespace

struct ihipStream_t;

namespace {

struct Op {
    OpKind k;
    void* dst = nullptr;
    const void* src = nullptr;
    size_t n = 0, dpitch = 0, spitch = 0, width = 0, height = 0;
    hipMemcpyKind kind = hipMemcpyDefault;
    ihipStream_t* wait = nullptr;   // OP_WAIT: the stream whose work comes first
    Site site;
};

}  // namespace

struct ihipGraph {
    std::vector<Op> ops;
};
struct hipGraphExec {
    std::vector<Op> ops;
};
struct ihipStream_t {
    std::deque<Op> q;
    unsigned flags = 0;
    ihipGraph* cap = nullptr;   // the graph this stream records into
    bool origin = false;        // capture began on this stream
    bool flushing = false;
};
struct ihipEvent_t {
    ihipStream_t* s = nullptr;
    ihipGraph* cap = nullptr;
    bool recorded = false;
};

namespace {

struct DevRange {
    size_t size;
    size_t map;
    bool freed;
};

struct State {
    std::recursive_mutex mu;
    std::map<uintptr_t, DevRange> dev;        // device allocations by base
    size_t allocated = 0;
    std::map<uintptr_t, size_t> pinned;       // hipHostMalloc blocks
    std::map<const void*, void*> symbols;     // host shadow -> device copy
    std::map<const void*, const char*> funcs; // registered kernels
    std::map<const void*, int> lds_attr;      // hipFuncSetAttribute values
    std::set<ihipStream_t*> streams;
    std::set<ihipEvent_t*> events;
    std::set<ihipGraph*> graphs;
    std::set<hipGraphExec*> execs;
    ihipStream_t null_stream;
    int capturing = 0;
};

State& st() {
    static State* s = new State;   // constructed on first use: kernels register from static constructors
    return *s;
}

#define LOCK std::lock_guard<std::recursive_mutex> lk_(st().mu)

hipError_t g_last = hipSuccess;   // sticky error of the last failed launch
long g_fail_at = -1;              // -1: not read yet, 0: off
long g_calls = 0;

long g_fail_site = 0;             // HOSTCHECK_FAIL_SITE: k-th distinct call site
std::vector<uint64_t>* g_sites = nullptr;

// Distinct call site of a fallible call: its callers' return addresses.
uint64_t site_key(const char* who) {
    void* pc[8];
    const int n = backtrace(pc, 8);
    uint64_t h = 1469598103934665603ull ^ reinterpret_cast<uintptr_t>(who);
    for (int i = 2; i < n; ++i) h = (h ^ reinterpret_cast<uintptr_t>(pc[i])) * 1099511628211ull;
    return h;
}

// True when this fallible call is the one to fail.
bool inject(const char* who) {
    if (g_fail_at < 0) {
        const char* e = getenv("HOSTCHECK_FAIL_AT");
        g_fail_at = e ? atol(e) : 0;
        const char* f = getenv("HOSTCHECK_FAIL_SITE");
        g_fail_site = f ? atol(f) : 0;
        g_sites = new std::vector<uint64_t>;
    }
    ++g_calls;
    if (g_fail_at > 0 && g_calls == g_fail_at) {
        fprintf(stderr, "HOSTCHECK-INJECT: call %ld (%s) fails\n", g_calls, who);
        return true;
    }
    const uint64_t k = site_key(who);
    if (std::find(g_sites->begin(), g_sites->end(), k) == g_sites->end()) {
        g_sites->push_back(k);
        if (g_fail_site > 0 && (long)g_sites->size() == g_fail_site) {
            fprintf(stderr, "HOSTCHECK-INJECT: first call at site %ld (%s) fails\n", g_fail_site, who);
            return true;
        }
    }
    return false;
}

thread_local struct {
    dim3 grid, block;
    size_t shmem = 0;
    hipStream_t stream = nullptr;
    bool set = false;
} t_cfg;

// Device allocation containing p (live or freed), or nullptr.
std::pair<const uintptr_t, DevRange>* dev_of(const void* p) {
    auto& d = st().dev;
    auto it = d.upper_bound(reinterpret_cast<uintptr_t>(p));
    if (it == d.begin()) return nullptr;
    --it;
    if (reinterpret_cast<uintptr_t>(p) < it->first + it->second.map) return &*it;
    return nullptr;
}

// True if [p, p+n) is device memory (checked to lie in one live allocation),
// false if it is host memory.
bool is_dev(const void* p, size_t n, const Site* site, const char* what) {
    auto* d = dev_of(p);
    if (!d) return false;
    if (d->second.freed) fail(site, "%s %p lies in device memory freed earlier (allocation %p, %zu bytes)", what, p,
                              (void*)d->first, d->second.size);
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    if (a + n > d->first + d->second.size)
        fail(site, "%s [%p, +%zu) overruns the device allocation %p of %zu bytes", what, p, n, (void*)d->first,
             d->second.size);
    return true;
}

void set_prot(const void* p, size_t n, int prot) {
    if (n == 0) return;
    const uintptr_t a = reinterpret_cast<uintptr_t>(p) & ~(kPage - 1);
    const uintptr_t e = (reinterpret_cast<uintptr_t>(p) + n + kPage - 1) & ~(kPage - 1);
    if (mprotect(reinterpret_cast<void*>(a), e - a, prot) != 0) fail(nullptr, "mprotect failed");
}

void check_host(const void* p, size_t n, const Site* site, const char* what) {
    if (n == 0) return;
    if (!p) fail(site, "%s is NULL", what);
    if (__asan_region_is_poisoned(const_cast<void*>(p), n)) {
        if (site) site->print("host memory named by a queued copy is no longer valid; the copy was enqueued at:");
        // let the sanitizer describe the region (freed heap block, dead frame, ...)
        volatile char c = *reinterpret_cast<const volatile char*>(__asan_region_is_poisoned(const_cast<void*>(p), n));
        (void)c;
        fail(site, "%s [%p, +%zu) is poisoned host memory", what, p, n);
    }
}

void do_copy(void* dst, const void* src, size_t n, hipMemcpyKind kind, const Site* site) {
    if (n == 0) return;
    const bool dd = is_dev(dst, n, site, "copy destination");
    const bool sd = is_dev(src, n, site, "copy source");
    switch (kind) {
        case hipMemcpyHostToDevice:
            if (!dd || sd) fail(site, "HostToDevice copy %p <- %p: destination %s, source %s", dst, src,
                                dd ? "device" : "host", sd ? "device" : "host");
            break;
        case hipMemcpyDeviceToHost:
            if (dd || !sd) fail(site, "DeviceToHost copy %p <- %p: destination %s, source %s", dst, src,
                                dd ? "device" : "host", sd ? "device" : "host");
            break;
        case hipMemcpyDeviceToDevice:
            if (!dd || !sd) fail(site, "DeviceToDevice copy %p <- %p: destination %s, source %s", dst, src,
                                 dd ? "device" : "host", sd ? "device" : "host");
            break;
        case hipMemcpyHostToHost:
            if (dd || sd) fail(site, "HostToHost copy names device memory");
            break;
        default:
            break;
    }
    if (!dd) check_host(dst, n, site, "copy destination");
    if (!sd) check_host(src, n, site, "copy source");
    if (dd) set_prot(dst, n, PROT_READ | PROT_WRITE);
    if (sd) set_prot(src, n, PROT_READ | PROT_WRITE);
    std::memmove(dst, src, n);
    if (dd) set_prot(dst, n, PROT_NONE);
    if (sd) set_prot(src, n, PROT_NONE);
}

void do_copy2d(const Op& o) {
    for (size_t r = 0; r < o.height; ++r)
        do_copy(static_cast<uint8_t*>(o.dst) + r * o.dpitch, static_cast<const uint8_t*>(o.src) + r * o.spitch,
                o.width, o.kind, &o.site);
}

bool live_stream(ihipStream_t* s) { return s == &st().null_stream || st().streams.count(s); }

ihipStream_t* S(hipStream_t s, const char* who) {
    ihipStream_t* p = s ? s : &st().null_stream;
    if (!live_stream(p)) fail(nullptr, "%s: stream %p is not a live stream", who, (void*)s);
    return p;
}

void flush(ihipStream_t* s);

void exec(const Op& o) {
    switch (o.k) {
        case OP_COPY:
            do_copy(o.dst, o.src, o.n, o.kind, &o.site);
            break;
        case OP_COPY2D:
            do_copy2d(o);
            break;
        case OP_WAIT:
            if (live_stream(o.wait)) flush(o.wait);
            break;
        case OP_KERNEL:
            break;
    }
}

void flush(ihipStream_t* s) {
    if (s->flushing) return;
    s->flushing = true;
    while (!s->q.empty()) {
        Op o = s->q.front();
        s->q.pop_front();
        exec(o);
    }
    s->flushing = false;
}

void flush_all() {
    flush(&st().null_stream);
    for (ihipStream_t* s : std::vector<ihipStream_t*>(st().streams.begin(), st().streams.end())) flush(s);
}

// the null stream waits for (and is waited for by) blocking streams
void flush_blocking() {
    flush(&st().null_stream);
    for (ihipStream_t* s : std::vector<ihipStream_t*>(st().streams.begin(), st().streams.end()))
        if (!(s->flags & hipStreamNonBlocking)) flush(s);
}

void enqueue(ihipStream_t* s, Op o) {
    if (s->cap)
        s->cap->ops.push_back(o);
    else
        s->q.push_back(o);
}

void no_capture(const char* who) {
    if (st().capturing) fail(nullptr, "%s called while a stream captures (not allowed in this capture mode)", who);
}

}  // namespace

extern "C" {

// ---------------------------------------------------------------- registration
void** __hipRegisterFatBinary(const void*) {
    static void* module = nullptr;
    return &module;
}

void __hipUnregisterFatBinary(void**) {}

void __hipRegisterFunction(void**, const void* hostFunction, char*, const char* deviceName, unsigned int, uint3*,
                           uint3*, dim3*, dim3*, int*) {
    LOCK;
    st().funcs[hostFunction] = deviceName;
}

void __hipRegisterVar(void**, void* var, char*, char*, int, size_t size, int, int) {
    LOCK;
    const size_t map = (std::max<size_t>(size, 1) + kPage - 1) & ~(kPage - 1);
    void* p = mmap(nullptr, map, PROT_NONE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
    if (p == MAP_FAILED) fail(nullptr, "cannot reserve %zu bytes for a device variable", size);
    st().dev[reinterpret_cast<uintptr_t>(p)] = DevRange{size, map, false};
    st().symbols[var] = p;
}

hipError_t __hipPushCallConfiguration(dim3 grid, dim3 block, size_t shmem, hipStream_t stream) {
    t_cfg.grid = grid;
    t_cfg.block = block;
    t_cfg.shmem = shmem;
    t_cfg.stream = stream;
    t_cfg.set = true;
    return hipSuccess;
}

hipError_t __hipPopCallConfiguration(dim3* grid, dim3* block, size_t* shmem, hipStream_t* stream) {
    if (!t_cfg.set) fail(nullptr, "launch configuration popped without a push");
    *grid = t_cfg.grid;
    *block = t_cfg.block;
    *shmem = t_cfg.shmem;
    *stream = t_cfg.stream;
    t_cfg.set = false;
    return hipSuccess;
}

hipError_t hipLaunchKernel(const void* fn, dim3 grid, dim3 block, void** args, size_t shmem, hipStream_t stream) {
    LOCK;
    Op o;
    o.k = OP_KERNEL;
    o.site.capture();
    auto it = st().funcs.find(fn);
    if (it == st().funcs.end()) fail(&o.site, "launch of an unregistered kernel %p", fn);
    const uint64_t threads = (uint64_t)block.x * block.y * block.z;
    if (threads == 0 || threads > 1024)
        fail(&o.site, "kernel %s: block of %llu threads", it->second, (unsigned long long)threads);
    if (grid.x == 0 || grid.y == 0 || grid.z == 0)
        fail(&o.site, "kernel %s: empty grid (%u, %u, %u)", it->second, grid.x, grid.y, grid.z);
    if ((uint64_t)grid.x * block.x > 0xFFFFFFFFull || (uint64_t)grid.y * block.y > 0xFFFFFFFFull ||
        (uint64_t)grid.z * block.z > 0xFFFFFFFFull)
        fail(&o.site, "kernel %s: grid (%u, %u, %u) x block (%u, %u, %u) exceeds 2^32 work-items in a dimension",
             it->second, grid.x, grid.y, grid.z, block.x, block.y, block.z);
    if (shmem > kLdsMax) fail(&o.site, "kernel %s: %zu bytes of dynamic LDS", it->second, shmem);
    (void)args;
    if (inject("hipLaunchKernel")) {
        g_last = hipErrorLaunchFailure;
        return hipErrorLaunchFailure;
    }
    enqueue(S(stream, "hipLaunchKernel"), o);
    return hipSuccess;
}

hipError_t hipFuncSetAttribute(const void* func, hipFuncAttribute attr, int value) {
    LOCK;
    if (!st().funcs.count(func)) fail(nullptr, "hipFuncSetAttribute on an unregistered kernel");
    if (attr == hipFuncAttributeMaxDynamicSharedMemorySize && (value < 0 || (size_t)value > kLdsMax))
        return hipErrorInvalidValue;
    st().lds_attr[func] = value;
    return hipSuccess;
}

hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, const void* f, int block, size_t dyn) {
    LOCK;
    if (!st().funcs.count(f)) fail(nullptr, "occupancy query on an unregistered kernel");
    if (block <= 0 || block > 1024) return hipErrorInvalidValue;
    const int waves = (block + 63) / 64;
    int by_waves = 32 / waves;
    int by_lds = dyn ? (int)(kLdsMax / dyn) : by_waves;
    *n = std::max(0, std::min(by_waves, by_lds));
    return hipSuccess;
}

// ---------------------------------------------------------------- device
hipError_t hipGetDevice(int* d) {
    *d = 0;
    return hipSuccess;
}

hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidDevice; }

hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_tR0600* p, int d) {
    if (d != 0) return hipErrorInvalidDevice;
    std::memset(p, 0, sizeof *p);
    std::snprintf(p->name, sizeof p->name, "host stand-in");
    std::snprintf(p->gcnArchName, sizeof p->gcnArchName, "gfx950:sramecc+:xnack-");
    p->multiProcessorCount = kCus;
    p->sharedMemPerBlock = 64 * 1024;
    p->maxSharedMemoryPerMultiProcessor = kLdsMax;
    p->totalGlobalMem = kHbm;
    p->warpSize = 64;
    p->maxThreadsPerBlock = 1024;
    p->clockRate = 2400000;
    p->l2CacheSize = 4 << 20;
    return hipSuccess;
}

hipError_t hipDeviceSynchronize() {
    LOCK;
    no_capture("hipDeviceSynchronize");
    flush_all();
    return hipSuccess;
}

hipError_t hipGetLastError() {
    hipError_t e = g_last;
    g_last = hipSuccess;
    return e;
}

hipError_t hipPeekAtLastError() { return g_last; }

const char* hipGetErrorString(hipError_t e) {
    switch (e) {
        case hipSuccess: return "no error";
        case hipErrorInvalidValue: return "invalid argument";
        case hipErrorOutOfMemory: return "out of memory";
        case hipErrorInvalidDevice: return "invalid device ordinal";
        case hipErrorInvalidSymbol: return "invalid device symbol";
        default: return "hip error (host stand-in)";
    }
}

const char* hipGetErrorName(hipError_t e) { return hipGetErrorString(e); }

// ---------------------------------------------------------------- memory
hipError_t hipMalloc(void** p, size_t size) {
    LOCK;
    no_capture("hipMalloc");
    if (!p) return hipErrorInvalidValue;
    if (size == 0) {
        *p = nullptr;
        return hipSuccess;
    }
    if (st().allocated + size > kHbm || inject("hipMalloc")) return hipErrorOutOfMemory;
    const size_t map = (size + kPage - 1) & ~(kPage - 1);
    void* m = mmap(nullptr, map, PROT_NONE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
    if (m == MAP_FAILED) return hipErrorOutOfMemory;
    st().dev[reinterpret_cast<uintptr_t>(m)] = DevRange{size, map, false};
    st().allocated += size;
    *p = m;
    return hipSuccess;
}

hipError_t hipFree(void* p) {
    LOCK;
    no_capture("hipFree");
    if (!p) return hipSuccess;
    flush_all();   // hipFree waits for the device
    auto it = st().dev.find(reinterpret_cast<uintptr_t>(p));
    if (it == st().dev.end()) fail(nullptr, "hipFree(%p): not the base of a device allocation", p);
    if (it->second.freed) fail(nullptr, "hipFree(%p): freed twice", p);
    it->second.freed = true;
    st().allocated -= it->second.size;
    madvise(p, it->second.map, MADV_DONTNEED);   // keep the range reserved, drop its pages
    return hipSuccess;
}

hipError_t hipMemGetInfo(size_t* free_b, size_t* total) {
    LOCK;
    *free_b = kHbm - st().allocated;
    *total = kHbm;
    return hipSuccess;
}

hipError_t hipHostMalloc(void** p, size_t size, unsigned int) {
    LOCK;
    no_capture("hipHostMalloc");
    if (inject("hipHostMalloc")) return hipErrorOutOfMemory;
    void* m = std::calloc(1, std::max<size_t>(size, 1));
    if (!m) return hipErrorOutOfMemory;
    st().pinned[reinterpret_cast<uintptr_t>(m)] = size;
    *p = m;
    return hipSuccess;
}

hipError_t hipHostFree(void* p) {
    LOCK;
    no_capture("hipHostFree");
    if (!p) return hipSuccess;
    flush_all();
    auto it = st().pinned.find(reinterpret_cast<uintptr_t>(p));
    if (it == st().pinned.end()) fail(nullptr, "hipHostFree(%p): not a hipHostMalloc block", p);
    st().pinned.erase(it);
    std::free(p);
    return hipSuccess;
}

hipError_t hipHostGetDevicePointer(void** d, void* h, unsigned int) {
    LOCK;
    auto& pm = st().pinned;
    auto it = pm.upper_bound(reinterpret_cast<uintptr_t>(h));
    if (it == pm.begin()) return hipErrorInvalidValue;
    --it;
    if (reinterpret_cast<uintptr_t>(h) >= it->first + it->second) return hipErrorInvalidValue;
    *d = h;
    return hipSuccess;
}

hipError_t hipGetSymbolAddress(void** d, const void* sym) {
    LOCK;
    auto it = st().symbols.find(sym);
    if (it == st().symbols.end()) return hipErrorInvalidSymbol;
    *d = it->second;
    return hipSuccess;
}

hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind kind) {
    LOCK;
    no_capture("hipMemcpy");
    if (inject("hipMemcpy")) return hipErrorInvalidValue;
    flush_blocking();
    Site s;
    s.capture();
    do_copy(dst, src, n, kind, &s);
    return hipSuccess;
}

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind kind, hipStream_t stream) {
    LOCK;
    Op o;
    o.k = OP_COPY;
    o.dst = dst;
    o.src = src;
    o.n = n;
    o.kind = kind;
    o.site.capture();
    if (n) {   // pointers are validated when the call is made, as the runtime does
        (void)is_dev(dst, n, &o.site, "copy destination");
        (void)is_dev(src, n, &o.site, "copy source");
    }
    if (inject("hipMemcpyAsync")) return hipErrorInvalidValue;
    enqueue(S(stream, "hipMemcpyAsync"), o);
    return hipSuccess;
}

hipError_t hipMemcpy2DAsync(void* dst, size_t dpitch, const void* src, size_t spitch, size_t width, size_t height,
                            hipMemcpyKind kind, hipStream_t stream) {
    LOCK;
    if (width > dpitch || width > spitch) return hipErrorInvalidValue;
    Op o;
    o.k = OP_COPY2D;
    o.dst = dst;
    o.src = src;
    o.dpitch = dpitch;
    o.spitch = spitch;
    o.width = width;
    o.height = height;
    o.kind = kind;
    o.site.capture();
    if (inject("hipMemcpy2DAsync")) return hipErrorInvalidValue;
    enqueue(S(stream, "hipMemcpy2DAsync"), o);
    return hipSuccess;
}

hipError_t hipMemset(void* dst, int v, size_t n) {
    LOCK;
    no_capture("hipMemset");
    if (inject("hipMemset")) return hipErrorInvalidValue;
    flush_blocking();
    if (n == 0) return hipSuccess;
    Site s;
    s.capture();
    if (!is_dev(dst, n, &s, "hipMemset destination")) fail(&s, "hipMemset of host memory %p", dst);
    set_prot(dst, n, PROT_READ | PROT_WRITE);
    std::memset(dst, v, n);
    set_prot(dst, n, PROT_NONE);
    return hipSuccess;
}

// ---------------------------------------------------------------- streams
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int flags) {
    LOCK;
    if (inject("hipStreamCreateWithFlags")) return hipErrorOutOfMemory;
    auto* p = new ihipStream_t;
    p->flags = flags;
    st().streams.insert(p);
    *s = p;
    return hipSuccess;
}

hipError_t hipStreamCreate(hipStream_t* s) { return hipStreamCreateWithFlags(s, 0); }

hipError_t hipStreamDestroy(hipStream_t s) {
    LOCK;
    if (!s || !st().streams.count(s)) fail(nullptr, "hipStreamDestroy(%p): not a live stream", (void*)s);
    if (s->cap && s->origin) fail(nullptr, "hipStreamDestroy of a stream that is capturing");
    flush(s);
    st().streams.erase(s);
    delete s;
    return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t s) {
    LOCK;
    no_capture("hipStreamSynchronize");
    ihipStream_t* p = S(s, "hipStreamSynchronize");
    if (inject("hipStreamSynchronize")) {   // as a kernel fault would be reported
        if (p == &st().null_stream)
            flush_blocking();
        else
            flush(p);
        return hipErrorLaunchFailure;
    }
    if (p == &st().null_stream)
        flush_blocking();
    else
        flush(p);
    return hipSuccess;
}

hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int) {
    LOCK;
    ihipStream_t* p = S(s, "hipStreamWaitEvent");
    if (!e || !st().events.count(e)) fail(nullptr, "hipStreamWaitEvent: %p is not a live event", (void*)e);
    if (e->cap) {
        if (p->cap && p->cap != e->cap) fail(nullptr, "hipStreamWaitEvent joins two different captures");
        p->cap = e->cap;   // the stream joins the capture
        return hipSuccess;
    }
    if (p->cap) return hipSuccess;   // an external dependency of the graph: nothing to record
    if (e->recorded && e->s) {
        Op o;
        o.k = OP_WAIT;
        o.wait = e->s;
        enqueue(p, o);
    }
    return hipSuccess;
}

hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    LOCK;
    ihipStream_t* p = S(s, "hipStreamBeginCapture");
    if (p == &st().null_stream) fail(nullptr, "capture on the null stream");
    if (p->cap) fail(nullptr, "hipStreamBeginCapture on a stream that already captures");
    if (inject("hipStreamBeginCapture")) return hipErrorOutOfMemory;
    p->cap = new ihipGraph;
    p->origin = true;
    ++st().capturing;
    return hipSuccess;
}

hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
    LOCK;
    ihipStream_t* p = S(s, "hipStreamEndCapture");
    if (!p->cap || !p->origin) fail(nullptr, "hipStreamEndCapture on a stream that did not begin a capture");
    ihipGraph* gr = p->cap;
    for (ihipStream_t* o : st().streams)
        if (o->cap == gr) o->cap = nullptr;
    p->origin = false;
    --st().capturing;
    st().graphs.insert(gr);
    *g = gr;
    return hipSuccess;
}

// ---------------------------------------------------------------- events
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned int) {
    LOCK;
    if (inject("hipEventCreateWithFlags")) return hipErrorOutOfMemory;
    auto* p = new ihipEvent_t;
    st().events.insert(p);
    *e = p;
    return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* e) { return hipEventCreateWithFlags(e, 0); }

hipError_t hipEventDestroy(hipEvent_t e) {
    LOCK;
    if (!e || !st().events.count(e)) fail(nullptr, "hipEventDestroy(%p): not a live event", (void*)e);
    st().events.erase(e);
    delete e;
    return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    LOCK;
    if (!e || !st().events.count(e)) fail(nullptr, "hipEventRecord(%p): not a live event", (void*)e);
    ihipStream_t* p = S(s, "hipEventRecord");
    e->s = p;
    e->cap = p->cap;
    e->recorded = p->cap == nullptr;
    return hipSuccess;
}

hipError_t hipEventSynchronize(hipEvent_t e) {
    LOCK;
    no_capture("hipEventSynchronize");
    if (!e || !st().events.count(e)) fail(nullptr, "hipEventSynchronize(%p): not a live event", (void*)e);
    if (e->cap) fail(nullptr, "hipEventSynchronize on an event recorded during capture");
    if (e->recorded && live_stream(e->s)) flush(e->s);
    return hipSuccess;
}

hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
    LOCK;
    if (!st().events.count(a) || !st().events.count(b)) fail(nullptr, "hipEventElapsedTime: not live events");
    if (!a->recorded || !b->recorded) return hipErrorInvalidHandle;
    *ms = 1.0f;
    return hipSuccess;
}

// ---------------------------------------------------------------- graphs
hipError_t hipGraphInstantiate(hipGraphExec_t* out, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
    LOCK;
    if (!g || !st().graphs.count(g)) fail(nullptr, "hipGraphInstantiate: %p is not a live graph", (void*)g);
    if (inject("hipGraphInstantiate")) return hipErrorOutOfMemory;
    auto* x = new hipGraphExec;
    x->ops = g->ops;
    st().execs.insert(x);
    *out = x;
    return hipSuccess;
}

hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
    LOCK;
    if (!x || !st().execs.count(x)) fail(nullptr, "hipGraphLaunch: %p is not a live executable graph", (void*)x);
    ihipStream_t* p = S(s, "hipGraphLaunch");
    if (inject("hipGraphLaunch")) return hipErrorInvalidValue;
    for (const Op& o : x->ops) {
        if (o.k == OP_WAIT) continue;
        if (o.n || o.height) {   // pointers must still be valid when the graph is launched
            if (o.k == OP_COPY) {
                (void)is_dev(o.dst, o.n, &o.site, "graph copy destination");
                (void)is_dev(o.src, o.n, &o.site, "graph copy source");
            }
        }
        enqueue(p, o);
    }
    return hipSuccess;
}

hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
    LOCK;
    if (!x || !st().execs.count(x)) fail(nullptr, "hipGraphExecDestroy(%p): not live", (void*)x);
    st().execs.erase(x);
    delete x;
    return hipSuccess;
}

hipError_t hipGraphDestroy(hipGraph_t g) {
    LOCK;
    if (!g || !st().graphs.count(g)) fail(nullptr, "hipGraphDestroy(%p): not live", (void*)g);
    st().graphs.erase(g);
    delete g;
    return hipSuccess;
}

// ---------------------------------------------------------------- test hooks
// Fallible calls made so far (the range of HOSTCHECK_FAIL_AT).
long hostcheck_calls() {
    LOCK;
    return g_calls;
}

// Distinct call sites of fallible calls so far (the range of HOSTCHECK_FAIL_SITE).
long hostcheck_sites() {
    LOCK;
    return g_sites ? (long)g_sites->size() : 0;
}

// Bytes of device memory live now (the harness checks that releases return it).
size_t hostcheck_device_bytes() {
    LOCK;
    return st().allocated;
}

}  // extern "C"
