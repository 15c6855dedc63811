// host_common.h -- host-side declarations shared by the C-ABI translation
// units of libpchase (workspace, validation, kernel launchers).
#pragma once

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace pc {

// ----------------------------------------------------------- validation --
int check_model(const pchase_model& m, DevModel* d, uint64_t index);
int check_probe(const pchase_probe& p, DevProbe* d, uint64_t* len, uint64_t index);

// ----------------------------------------------------------- workspace ---
// Device memory reserved once (by a caller-owned pchase_plan): buffers are
// carved from it front to back and never freed one by one; reset() makes
// the whole of it available again.
struct Arena {
    uint8_t* base = nullptr;
    size_t cap = 0, used = 0;
    void reset() { used = 0; }
};

// Growable device buffer: its own hipMalloc, or a block carved from an
// arena (then ensure() fails with hipErrorOutOfMemory instead of
// allocating when the arena is used up).
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    Arena* arena = nullptr;
    hipError_t ensure(size_t n);
    void release();
    template <class T>
    T* as() const { return static_cast<T*>(p); }
};

struct InferPlan;

// Streams of a concurrent launch sequence: the caller's stream and three
// workspace streams, one per hardware queue of the process (the runtime's
// default of four queues; a fifth stream would share a queue with another
// and its kernels would wait for that stream's).
constexpr int kBranches = 4;

struct Workspace {
    int device = -1;
    int cus = 0;
    std::mutex mu;
    DevBuf stage;      // per-call descriptors
    DevBuf aux;        // per-call device scratch (counters, queues, results)
    DevBuf obs;        // derived observed bitmaps
    DevBuf slab;       // stream-replay set state
    DevBuf mlp;        // grid replay bank of the learned proposer
    DevBuf gsearch;    // generalised-candidate search: traces, hit bits, scores
    size_t slab_clean = 0;  // bytes of `slab` known to hold epoch 0 or older epochs
    uint32_t epoch = 0;
    void* host_res = nullptr;  // pinned result staging
    int occ_stream[2][5][7] = {};   // [generalised][policy][log2 width]
    int occ_tile[4 * 5][8] = {};    // [policy * way classes + way class][log2 row class - 4]
    bool tile_ready = false;
    bool lds_ready = false;
    // branch streams of a batched sweep beyond the caller's own (default priority)
    hipStream_t branch[kBranches - 1] = {};
    hipEvent_t fork = nullptr, join[kBranches - 1] = {};
    std::map<std::string, std::unique_ptr<InferPlan>> plans;
    // the last one-off inference plan (the learned proposer's confirmation):
    // its device buffers serve the next one, which grows them only when
    // needed (not with an arena)
    std::unique_ptr<InferPlan> oneoff;
    // probe planner: class matrix of the last (candidates, pool) pair
    DevBuf planner;
    std::string planner_key;
    // set for the workspace of a caller-owned plan: every device buffer
    // comes from this arena
    Arena* arena = nullptr;
    // forgets every buffer and cached schedule carved from the arena
    void reset_arena();
    ~Workspace();
};

// Guards host memory that queued copies read: declared after the host
// buffers of a scope and before its first asynchronous copy out of them, it
// makes any return that has not synchronised `stream` (an error return)
// wait for the stream before those buffers are destroyed, so that no copy
// still in the queue reads freed memory.  done() once the scope has
// synchronised the stream itself.
struct CopyFence {
    hipStream_t stream;
    bool armed = true;
    explicit CopyFence(hipStream_t s) : stream(s) {}
    CopyFence(const CopyFence&) = delete;
    CopyFence& operator=(const CopyFence&) = delete;
    ~CopyFence() {
        if (armed) (void)hipStreamSynchronize(stream);
    }
    void done() { armed = false; }
};

// Branch b of a concurrent sequence on `s`: `s` itself for b = 0, else
// workspace stream b - 1.
inline hipStream_t branch_stream(Workspace* ws, hipStream_t s, int b) { return b == 0 ? s : ws->branch[b - 1]; }
// Branches 1 .. n-1 wait for the work enqueued on `s` so far.
hipError_t fork_branches(Workspace* ws, hipStream_t s, int n);
// `s` waits for the work enqueued on branches 1 .. n-1.
hipError_t join_branches(Workspace* ws, hipStream_t s, int n);

// Locks and returns the calling thread's current device's workspace.
int workspace(Workspace** ws, std::unique_lock<std::mutex>* lock);
// The plan's workspace when plan is not NULL (checked against the current
// device), else the device's own.
int workspace_for(pchase_plan* plan, Workspace** ws, std::unique_lock<std::mutex>* lock);
// Creates the streams, events and pinned result page of a workspace.
int workspace_init(Workspace* ws);
const volatile uint32_t* abort_flag_dev();
uint32_t abort_flag_host();


}  // namespace pc
