// runtime.hip -- host runtime of libpchase: error reporting, per-device
// workspace, argument validation, persistent-grid sizing.
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "host_common.h"
#include "plan.h"

namespace pc {

// ---------------------------------------------------------------- errors --
static thread_local std::string g_last_error;

int set_error(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return set_error(PCHASE_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// ----------------------------------------------------------- validation --
static bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }
static uint32_t ilog2(uint64_t x) {
    uint32_t r = 0;
    while (x > 1) {
        x >>= 1;
        ++r;
    }
    return r;
}
static uint64_t gcd64(uint64_t a, uint64_t b) {
    while (b) {
        uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

int check_model(const pchase_model& m, DevModel* d, uint64_t i) {
    if (m.reserved != 0) return set_error(PCHASE_EINVAL, "model %llu: reserved field must be 0", (unsigned long long)i);
    if (m.ways == 0 || m.sets == 0) return set_error(PCHASE_EINVAL, "model %llu: ways and sets must be >= 1", (unsigned long long)i);
    if (m.line_bytes < 4 || !is_pow2(m.line_bytes))
        return set_error(PCHASE_EINVAL, "model %llu: line_bytes %u is not a power of two >= 4", (unsigned long long)i, m.line_bytes);
    if ((uint64_t)m.sets * m.ways * m.line_bytes != m.capacity_bytes)
        return set_error(PCHASE_EINVAL, "model %llu: sets*ways*line_bytes != capacity_bytes (Assumption 1)", (unsigned long long)i);
    if (m.policy > PCHASE_RANDOM) return set_error(PCHASE_EINVAL, "model %llu: unknown policy %u", (unsigned long long)i, m.policy);
    if (m.policy == PCHASE_PLRU && !is_pow2(m.ways))
        return set_error(PCHASE_EINVAL, "model %llu: tree-PLRU needs a power-of-two associativity", (unsigned long long)i);
    const uint32_t ls = ilog2(m.line_bytes);
    if (m.set_shift != 0 && (m.set_shift < ls || m.set_shift > 40))
        return set_error(PCHASE_EINVAL, "model %llu: set_shift must be 0 or in [log2(line_bytes), 40]", (unsigned long long)i);
    if (m.ways > kMaxWays) return set_error(PCHASE_ERANGE, "model %llu: ways %u above the supported 128", (unsigned long long)i, m.ways);
    if (d) {
        d->line_shift = ls;
        d->unit_shift = m.set_shift ? m.set_shift : ls;
        d->sets = m.sets;
        d->ways = m.ways;
        d->policy = m.policy;
        d->log2_ways = ilog2(m.ways);
        d->seed_lo = (uint32_t)m.seed;
        d->seed_hi = (uint32_t)(m.seed >> 32);
    }
    return PCHASE_OK;
}

int check_probe(const pchase_probe& p, DevProbe* d, uint64_t* len, uint64_t i) {
    if (p.elem_bytes != 4) return set_error(PCHASE_EINVAL, "probe %llu: elem_bytes must be 4", (unsigned long long)i);
    if (p.n_bytes == 0 || p.n_bytes % 4 || p.s_bytes % 4)
        return set_error(PCHASE_EINVAL, "probe %llu: N and s must be positive multiples of elem_bytes", (unsigned long long)i);
    const uint64_t ne = p.n_bytes / 4;
    if (ne >= (1ull << 31)) return set_error(PCHASE_EINVAL, "probe %llu: N/elem must be below 2^31", (unsigned long long)i);
    if (p.j0 >= ne) return set_error(PCHASE_EINVAL, "probe %llu: j0 outside the array", (unsigned long long)i);
    if (p.passes == 0) return set_error(PCHASE_EINVAL, "probe %llu: passes must be >= 1", (unsigned long long)i);
    if (p.base_offset >= (1ull << 33) || p.base_offset % 4)
        return set_error(PCHASE_EINVAL, "probe %llu: base_offset must be a multiple of 4 below 2^33", (unsigned long long)i);
    const uint64_t se = (p.s_bytes / 4) % ne;
    const uint64_t L = ne / gcd64(ne, se);
    if (L * (uint64_t)p.passes >= (1ull << 32))
        return set_error(PCHASE_ERANGE, "probe %llu: passes * cycle length must stay below 2^32 accesses", (unsigned long long)i);
    if (len) *len = L * p.passes;
    if (d) {
        d->base = p.base_offset;
        d->ne = (uint32_t)ne;
        d->se = (uint32_t)se;
        d->L = (uint32_t)L;
        d->j0 = (uint32_t)p.j0;
        d->passes = p.passes;
        d->elem_shift = 2;
        const uint64_t sb = se * 4;
        d->sb_fast = (sb > 0 && sb < (1ull << 32)) ? 1u : 0u;
        d->sb_div = make_udiv32(d->sb_fast ? (uint32_t)sb : 1u);
    }
    return PCHASE_OK;
}

// ------------------------------------------------------------ workspace --
hipError_t DevBuf::ensure(size_t n) {
    if (n <= cap) return hipSuccess;
    if (arena) {
        const size_t at = (arena->used + 255) / 256 * 256;
        if (at > arena->cap || n > arena->cap - at) {
            p = nullptr;
            cap = 0;
            return hipErrorOutOfMemory;
        }
        p = arena->base + at;
        cap = n;
        arena->used = at + n;
        return hipSuccess;
    }
    size_t want = cap ? cap : 1 << 20;
    while (want < n) want *= 2;
    if (p) {
        hipError_t e = hipFree(p);
        p = nullptr;
        cap = 0;
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        p = nullptr;
        return e;
    }
    cap = want;
    return hipSuccess;
}

void DevBuf::release() {
    if (p && !arena) (void)hipFree(p);
    p = nullptr;
    cap = 0;
}

void Workspace::reset_arena() {
    if (!arena) return;
    plans.clear();
    oneoff.reset();
    planner_key.clear();
    for (DevBuf* b : {&stage, &aux, &obs, &slab, &mlp, &planner, &gsearch}) b->release();
    slab_clean = 0;
    arena->reset();
}

Workspace::~Workspace() {
    for (int b = 0; b < kBranches - 1; ++b) {
        if (branch[b]) (void)hipStreamDestroy(branch[b]);
        if (join[b]) (void)hipEventDestroy(join[b]);
    }
    if (fork) (void)hipEventDestroy(fork);
    stage.release();
    aux.release();
    obs.release();
    slab.release();
    mlp.release();
    planner.release();
    gsearch.release();
    if (host_res) (void)hipHostFree(host_res);
}

hipError_t fork_branches(Workspace* ws, hipStream_t s, int n) {
    if (n < 2) return hipSuccess;
    hipError_t e = hipEventRecord(ws->fork, s);
    for (int b = 1; b < n && e == hipSuccess; ++b) e = hipStreamWaitEvent(ws->branch[b - 1], ws->fork, 0);
    return e;
}

hipError_t join_branches(Workspace* ws, hipStream_t s, int n) {
    hipError_t e = hipSuccess;
    for (int b = 1; b < n && e == hipSuccess; ++b) {
        e = hipEventRecord(ws->join[b - 1], ws->branch[b - 1]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, ws->join[b - 1], 0);
    }
    return e;
}

static std::mutex g_ws_mu;
static std::map<int, std::unique_ptr<Workspace>> g_ws;

int workspace(Workspace** out, std::unique_lock<std::mutex>* lock) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(PCHASE_ENODEV, "no HIP device: %s", hipGetErrorString(e));
    Workspace* ws;
    {
        std::lock_guard<std::mutex> g(g_ws_mu);
        auto& slot = g_ws[dev];
        if (!slot) {
            hipDeviceProp_t prop;
            e = hipGetDeviceProperties(&prop, dev);
            if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
            if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
                return set_error(PCHASE_ENODEV, "device %d is %s, the library is built for gfx950", dev,
                                 prop.gcnArchName);
            slot.reset(new Workspace());
            slot->device = dev;
            slot->cus = prop.multiProcessorCount;
        }
        ws = slot.get();
    }
    *lock = std::unique_lock<std::mutex>(ws->mu);
    int rc = workspace_init(ws);
    if (rc) return rc;
    *out = ws;
    return PCHASE_OK;
}

int workspace_init(Workspace* ws) {
    hipError_t e;
    if (!ws->host_res) {
        e = hipHostMalloc(&ws->host_res, 4096, hipHostMallocDefault);
        if (e != hipSuccess) {
            ws->host_res = nullptr;
            return hip_fail(e, "hipHostMalloc");
        }
    }
    if (abort_flag_dev() == nullptr) return set_error(PCHASE_ENOMEM, "mapped host flag allocation failed");
    if (!ws->lds_ready) {
        e = sweep_prepare_lds();
        if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
        for (int b = 0; b < kBranches - 1; ++b) {
            e = hipStreamCreateWithFlags(&ws->branch[b], hipStreamNonBlocking);
            if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
            e = hipEventCreateWithFlags(&ws->join[b], hipEventDisableTiming);
            if (e != hipSuccess) return hip_fail(e, "hipEventCreateWithFlags");
        }
        e = hipEventCreateWithFlags(&ws->fork, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreateWithFlags");
        ws->lds_ready = true;
    }
    return PCHASE_OK;
}

// A host flag, visible to kernels through a mapped pinned page.
static std::mutex g_abort_mu;
static volatile uint32_t* g_abort_host = nullptr;
static const volatile uint32_t* g_abort_dev = nullptr;

const volatile uint32_t* abort_flag_dev() {
    std::lock_guard<std::mutex> g(g_abort_mu);
    if (!g_abort_host) {
        void* h = nullptr;
        if (hipHostMalloc(&h, 64, hipHostMallocMapped | hipHostMallocPortable) != hipSuccess) return nullptr;
        std::memset(h, 0, 64);
        void* d = nullptr;
        if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) return nullptr;
        g_abort_host = static_cast<volatile uint32_t*>(h);
        g_abort_dev = static_cast<const volatile uint32_t*>(d);
    }
    return g_abort_dev;
}

uint32_t abort_flag_host() { return g_abort_host ? *g_abort_host : 0; }

}  // namespace pc

// A caller-owned plan: its own workspace over one device allocation.
struct pchase_plan {
    int device = -1;
    void* mem = nullptr;
    pc::Arena arena;
    pc::Workspace ws;
};

namespace pc {

int workspace_for(pchase_plan* plan, Workspace** out, std::unique_lock<std::mutex>* lock) {
    if (!plan) return workspace(out, lock);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(PCHASE_ENODEV, "no HIP device: %s", hipGetErrorString(e));
    if (dev != plan->device)
        return set_error(PCHASE_EINVAL, "the plan belongs to device %d, the current device is %d", plan->device, dev);
    *lock = std::unique_lock<std::mutex>(plan->ws.mu);
    *out = &plan->ws;
    return PCHASE_OK;
}

}  // namespace pc

extern "C" int pchase_plan_create(uint64_t device_bytes, pchase_plan** out) {
    using namespace pc;
    if (!out) return set_error(PCHASE_EINVAL, "out is NULL");
    *out = nullptr;
    if (device_bytes == 0) return set_error(PCHASE_EINVAL, "a plan needs device memory (device_bytes = 0)");
    Workspace* dws;
    std::unique_lock<std::mutex> lk;
    int rc = workspace(&dws, &lk);   // checks the device, creates the shared abort flag
    if (rc) return rc;
    const int dev = dws->device, cus = dws->cus;
    lk.unlock();
    std::unique_ptr<pchase_plan> p(new pchase_plan());
    p->device = dev;
    hipError_t e = hipMalloc(&p->mem, device_bytes);
    if (e != hipSuccess) {
        p->mem = nullptr;
        return set_error(PCHASE_ENOMEM, "plan memory of %llu bytes: %s", (unsigned long long)device_bytes,
                         hipGetErrorString(e));
    }
    p->arena.base = static_cast<uint8_t*>(p->mem);
    p->arena.cap = device_bytes;
    p->ws.device = dev;
    p->ws.cus = cus;
    p->ws.arena = &p->arena;
    for (DevBuf* b : {&p->ws.stage, &p->ws.aux, &p->ws.obs, &p->ws.slab, &p->ws.mlp, &p->ws.planner,
                       &p->ws.gsearch})
        b->arena = &p->arena;
    rc = workspace_init(&p->ws);
    if (rc) {
        pchase_plan_destroy(p.release());
        return rc;
    }
    *out = p.release();
    return PCHASE_OK;
}

extern "C" void pchase_plan_destroy(pchase_plan* plan) {
    if (!plan) return;
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    const int dev = plan->device;
    if (have && cur != dev) (void)hipSetDevice(dev);
    (void)hipDeviceSynchronize();
    plan->ws.reset_arena();
    void* mem = plan->mem;
    delete plan;   // the workspace's streams, events and pinned page
    if (mem) (void)hipFree(mem);
    if (have && cur != dev) (void)hipSetDevice(cur);
}

// ------------------------------------------------------------- C ABI ----
extern "C" const char* pchase_last_error(void) { return pc::g_last_error.c_str(); }

extern "C" void pchase_abort(int on) {
    const volatile uint32_t* d = pc::abort_flag_dev();
    (void)d;
    if (pc::g_abort_host) *pc::g_abort_host = on ? 1u : 0u;
}

extern "C" int pchase_release(void) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return pc::set_error(PCHASE_ENODEV, "no HIP device");
    std::unique_ptr<pc::Workspace> victim;
    {
        std::lock_guard<std::mutex> g(pc::g_ws_mu);
        auto it = pc::g_ws.find(dev);
        if (it == pc::g_ws.end()) return PCHASE_OK;
        victim = std::move(it->second);
        pc::g_ws.erase(it);
    }
    if (victim) {
        std::lock_guard<std::mutex> g(victim->mu);
        (void)hipDeviceSynchronize();
    }
    return PCHASE_OK;
}

extern "C" int pchase_trace_len(const pchase_probe* probe, uint64_t* len, uint64_t* cycle) {
    if (!probe) return pc::set_error(PCHASE_EINVAL, "probe is NULL");
    pc::DevProbe d;
    uint64_t n = 0;
    int rc = pc::check_probe(*probe, &d, &n, 0);
    if (rc) return rc;
    if (len) *len = n;
    if (cycle) *cycle = d.L;
    return PCHASE_OK;
}
