// plan.hip -- building and running probe-replay schedules.
//
// A job is one replay (model, probe).  A model with T sets gives each job
// G = min(T, 64) lanes (lane g owns sets g, g+G, ...); a task is 64
// consecutive (job, lane) items of one model.  Tasks are grouped by
// (policy, way class) because each group is one kernel instantiation.
//
// PLAIN runs one ordinary launch per model, tasks in natural order.
// BATCHED runs one persistent launch per group, each wave pulling tasks
// from an atomic queue in longest-first order (a counting sort on a
// log-scale cost estimate), the groups spread over parallel branch streams.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "plan.h"
#include "sweep_lane.h"

namespace pc {

void Digest::add(const void* p, size_t n) {
    // eight bytes per step, two independent multiply-xorshift lanes
    const uint8_t* c = static_cast<const uint8_t*>(p);
    size_t i = 0;
    for (; i + 8 <= n; i += 8) {
        uint64_t w;
        std::memcpy(&w, c + i, 8);
        a = (a ^ w) * 0x9E3779B97F4A7C15ull;
        a ^= a >> 32;
        b = (b + w) * 0xFF51AFD7ED558CCDull;
        b ^= b >> 29;
    }
    uint64_t t = 0;
    for (size_t k = 0; i < n; ++i, ++k) t |= (uint64_t)c[i] << (8 * k);
    a = (a ^ t ^ n) * 0x9E3779B97F4A7C15ull;
    b = (b + t + n) * 0xC4CEB9FE1A85EC53ull;
    b ^= b >> 33;
}

std::string Digest::str() const {
    char buf[40];
    snprintf(buf, sizeof buf, "%016llx%016llx", (unsigned long long)a, (unsigned long long)b);
    return buf;
}

SweepPlan::~SweepPlan() { dev.release(); }

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int build_sweep_plan(SweepPlan* plan, const std::vector<DevModel>& models, const std::vector<DevProbe>& probes,
                     const std::vector<uint64_t>& probe_len, const std::vector<SweepJob>& jobs_in,
                     bool want_clear, bool lds_bitmaps) {
    plan->n_models = (uint32_t)models.size();
    plan->n_probes = (uint32_t)probes.size();
    plan->n_jobs = jobs_in.size();
    std::vector<SweepJob> jobs(jobs_in);

    // --- natural task order: per model run of jobs; a task holds whole jobs,
    // G lanes each (G chosen per model below)
    std::vector<SweepTask> tasks;
    std::vector<float> cost;
    std::vector<uint8_t> tcls;
    std::vector<uint16_t> tmap;   // map dwords a map-class task needs
    plan->plain.clear();
    plan->accesses = 0;
    size_t j = 0;
    while (j < jobs.size()) {
        const uint32_t mi = jobs[j].model;
        size_t e = j;
        while (e < jobs.size() && jobs[e].model == mi) ++e;
        const DevModel& m = models[mi];
        // closed-form jobs (scoring) first: each group forms tasks of its own
        const size_t mid = (size_t)(std::stable_partition(jobs.begin() + j, jobs.begin() + e,
                                                          [](const SweepJob& x) { return x.cyc != 0; }) -
                                    jobs.begin());
        for (int grp = 0; grp < 2; ++grp) {
            const size_t gb = grp == 0 ? j : mid, ge = grp == 0 ? mid : e;
            if (gb == ge) continue;
            // G lanes per job: the choice that keeps most lanes busy, counting
            // lanes left idle (64 mod G) and sets shared unevenly (T mod G), with
            // at most as many jobs per task as the LDS bitmap holds
            uint64_t maxw = 1;
            for (size_t q = gb; q < ge; ++q) maxw = std::max<uint64_t>(maxw, (probe_len[jobs[q].probe] + 31) / 32);
            const uint64_t jpt_bm = lds_bitmaps ? std::max<uint64_t>(1, kBmMaxWords / maxw) : kWave;
            const uint64_t T = m.sets;
            uint64_t G = std::min<uint64_t>(T, kWave);
            double best = -1;
            for (uint64_t d = std::min<uint64_t>(T, kWave); d >= 1; --d) {
                const uint64_t jp = std::min<uint64_t>(std::max<uint64_t>(1, kWave / d), jpt_bm);
                const double sets_per_lane = std::ceil((double)T / (double)d);
                const double eff = (double)(jp * d) / kWave * ((double)T / (double)d) / sets_per_lane;
                if (eff > best + 0.03) {
                    best = eff;
                    G = d;
                }
            }
            const uint64_t jpt = std::min<uint64_t>(std::max<uint64_t>(1, kWave / G), jpt_bm);  // jobs per task
            const double per_set = std::ceil((double)m.sets / (double)G) / (double)m.sets;
            const int base_cls = grp == 0 ? (int)kACyc : way_class(m.ways);
            for (uint64_t q0 = gb; q0 < ge; q0 += jpt) {
                const uint64_t q1 = std::min<uint64_t>(ge, q0 + jpt);
                SweepTask t;
                t.job = (uint32_t)gb;
                t.item0 = (uint32_t)((q0 - gb) * G);
                t.n = (uint32_t)((q1 - q0) * G);
                t.model = mi;
                t.lanes = (uint32_t)G;
                uint64_t ml = 0, me = 0, words = 0;
                for (uint64_t q = q0; q < q1; ++q) {
                    const uint64_t len = probe_len[jobs[q].probe];
                    ml = std::max(ml, len);
                    if (base_cls == kALds) me = std::max(me, map_entries(probes[jobs[q].probe], m));
                    jobs[q].bm_off = (uint32_t)words;
                    words += (len + 31) / 32;
                }
                t.bm_words = (lds_bitmaps && words <= kBmMaxWords) ? (uint32_t)words : 0u;
                int cls = base_cls;
                double wcost = 1.0;
                if (base_cls == kALds) {
                    if (me <= kMapMaxEntries) cls = kAMap;
                    else wcost = (double)m.ways;
                } else if (base_cls == kACyc) {
                    wcost = 0.5;   // the first pass only, no way state
                }
                tasks.push_back(t);
                tcls.push_back((uint8_t)cls);
                tmap.push_back((uint16_t)(cls == kAMap ? (me + 3) / 4 : 0));
                cost.push_back((float)((double)ml * per_set * wcost + 64.0));
            }
        }
        for (size_t q = j; q < e; ++q) plan->accesses += probe_len[jobs[q].probe];
        j = e;
    }
    plan->n_tasks = tasks.size();

    auto rows_of = [&](size_t i, uint32_t* lds_rows, uint32_t* map_rows) {
        const DevModel& m = models[tasks[i].model];
        if (tcls[i] == kAMap) {
            *map_rows = tmap[i];
            *lds_rows = map_class_rows(tmap[i], m.ways, (int)m.policy);
        } else if (tcls[i] == kALds) {
            *map_rows = 0;
            *lds_rows = m.ways + (m.ways + 3) / 4;
        } else {
            *map_rows = *lds_rows = 0;
        }
    };
    // plain launches: runs of tasks with one model and one class
    for (size_t i = 0; i < tasks.size(); ++i) {
        const DevModel& m = models[tasks[i].model];
        uint32_t lr, mr;
        rows_of(i, &lr, &mr);
        if (plan->plain.empty() || tasks[plan->plain.back().first].model != tasks[i].model ||
            plan->plain.back().cls != tcls[i])
            plan->plain.push_back(Bucket{(int)m.policy, (int)tcls[i], (uint32_t)i, 0, 0, 0, 0.0, 0});
        Bucket& b = plan->plain.back();
        b.count++;
        b.map_rows = std::max(b.map_rows, mr);
        b.bm_words = std::max(b.bm_words, tasks[i].bm_words);
    }
    for (Bucket& b : plan->plain)
        if (b.cls == kAMap || b.cls == kALds) {
            uint32_t amax = 0;
            for (uint32_t i = b.first; i < b.first + b.count; ++i) amax = std::max(amax, models[tasks[i].model].ways);
            b.lds_rows = b.cls == kAMap ? map_class_rows(b.map_rows, amax, b.pol) : amax + (amax + 3) / 4;
        }

    // --- batched order: group by (policy, class), longest first within a group
    std::vector<uint32_t> order(tasks.size());
    {
        // key = group * 256 + (255 - log-cost bucket); counting sort
        const int nkeys = 4 * kNumClasses * 256;
        std::vector<uint32_t> cnt(nkeys + 1, 0);
        std::vector<uint32_t> key(tasks.size());
        for (size_t i = 0; i < tasks.size(); ++i) {
            const DevModel& m = models[tasks[i].model];
            // closed-form tasks of LRU and FIFO models share one kernel
            const int pol = tcls[i] == kACyc ? (int)PCHASE_LRU : (int)m.policy;
            const int grp = pol * kNumClasses + tcls[i];
            int cb = (int)std::floor(std::log2((double)cost[i] + 1.0) * 8.0);
            cb = std::max(0, std::min(255, cb));
            key[i] = (uint32_t)(grp * 256 + (255 - cb));
            ++cnt[key[i] + 1];
        }
        for (int k = 0; k < nkeys; ++k) cnt[k + 1] += cnt[k];
        for (size_t i = 0; i < tasks.size(); ++i) order[cnt[key[i]]++] = (uint32_t)i;
    }
    std::vector<SweepTask> lpt(tasks.size());
    plan->batched.clear();
    std::vector<uint32_t> bucket_amax;
    for (size_t i = 0; i < order.size(); ++i) {
        lpt[i] = tasks[order[i]];
        const DevModel& m = models[lpt[i].model];
        const int cls = tcls[order[i]];
        const int pol = cls == kACyc ? (int)PCHASE_LRU : (int)m.policy;
        if (plan->batched.empty() || plan->batched.back().pol != pol || plan->batched.back().cls != cls) {
            plan->batched.push_back(Bucket{pol, cls, (uint32_t)i, 0, 0, 0, 0.0, 0});
            bucket_amax.push_back(0);
        }
        Bucket& b = plan->batched.back();
        b.count++;
        b.cost += cost[order[i]];
        b.bm_words = std::max(b.bm_words, lpt[i].bm_words);
        uint32_t lr, mr;
        rows_of(order[i], &lr, &mr);
        b.map_rows = std::max(b.map_rows, mr);
        bucket_amax.back() = std::max(bucket_amax.back(), m.ways);
    }
    for (size_t k = 0; k < plan->batched.size(); ++k) {
        Bucket& b = plan->batched[k];
        if (b.cls == kAMap) b.lds_rows = map_class_rows(b.map_rows, bucket_amax[k], b.pol);
        else if (b.cls == kALds) b.lds_rows = bucket_amax[k] + (bucket_amax[k] + 3) / 4;
    }

    // --- bitmap ranges each job writes
    plan->clear.clear();
    if (want_clear) {
        for (const SweepJob& jb : jobs) {
            plan->clear.push_back(jb.bitoff);
            plan->clear.push_back((probe_len[jb.probe] + 31) / 32);
        }
    }

    // --- one device allocation for everything
    size_t off = 0;
    const size_t o_models = off; off = align_up(off + models.size() * sizeof(DevModel), 256);
    const size_t o_probes = off; off = align_up(off + probes.size() * sizeof(DevProbe), 256);
    const size_t o_jobs = off; off = align_up(off + jobs.size() * sizeof(SweepJob), 256);
    const size_t o_lpt = off; off = align_up(off + lpt.size() * sizeof(SweepTask), 256);
    const size_t o_plain = off; off = align_up(off + tasks.size() * sizeof(SweepTask), 256);
    const size_t o_queues = off; off = align_up(off + (plan->batched.size() + 2) * sizeof(uint32_t), 256);
    const size_t o_clear = off; off = align_up(off + plan->clear.size() * sizeof(uint64_t), 256);
    hipError_t e = plan->dev.ensure(off);
    if (e != hipSuccess) {
        if (plan->dev.arena)
            return set_error(PCHASE_ERANGE, "a replay schedule of %zu bytes does not fit the plan's device memory", off);
        return set_error(PCHASE_ENOMEM, "schedule allocation of %zu bytes: %s", off, hipGetErrorString(e));
    }
    uint8_t* base = plan->dev.as<uint8_t>();
    plan->d_models = reinterpret_cast<DevModel*>(base + o_models);
    plan->d_probes = reinterpret_cast<DevProbe*>(base + o_probes);
    plan->d_jobs = reinterpret_cast<SweepJob*>(base + o_jobs);
    plan->d_lpt = reinterpret_cast<SweepTask*>(base + o_lpt);
    plan->d_plain = reinterpret_cast<SweepTask*>(base + o_plain);
    plan->d_queues = reinterpret_cast<uint32_t*>(base + o_queues);
    plan->d_clear = reinterpret_cast<uint64_t*>(base + o_clear);
    // one upload of the whole block from a host image of it (the queues are
    // cleared by every run)
    std::vector<uint8_t> img(off, 0);
    auto put = [&](size_t at, const void* src, size_t n) {
        if (n) std::memcpy(img.data() + at, src, n);
    };
    put(o_models, models.data(), models.size() * sizeof(DevModel));
    put(o_probes, probes.data(), probes.size() * sizeof(DevProbe));
    put(o_jobs, jobs.data(), jobs.size() * sizeof(SweepJob));
    put(o_lpt, lpt.data(), lpt.size() * sizeof(SweepTask));
    put(o_plain, tasks.data(), tasks.size() * sizeof(SweepTask));
    put(o_clear, plan->clear.data(), plan->clear.size() * sizeof(uint64_t));
    PC_HIP(hipMemcpy(base, img.data(), off, hipMemcpyHostToDevice));
    return PCHASE_OK;
}

// Enqueues the batched sequence on `s`: the buckets, one persistent kernel
// each, are spread over parallel branch streams (least-loaded branch first,
// largest bucket first) so that one bucket's tail overlaps the next
// bucket's work; the branches join `s` again before the tail.
// Branch assignment strategies the autotuner tries (strategy 0 is the
// untuned default): 0 greedy over 4 branches by estimated cost; 1 the same
// with LDS-class buckets weighted 3x (their occupancy is LDS-bound); 2 greedy
// over 2 branches; 3 one branch; 4 LDS-class buckets each on a branch of
// their own first, then the rest greedily.
constexpr int kStrategies = 5;

static int enqueue_batched(Workspace* ws, SweepPlan* plan, bool score, uint64_t* counters,
                           uint64_t n_counters, uint32_t* bits, bool clear_bits, hipStream_t s,
                           const std::function<hipError_t(hipStream_t)>& tail,
                           const std::function<hipError_t(hipStream_t)>& side, int strategy = 0) {
    const uint32_t nq = (uint32_t)plan->batched.size() + 2;
    PC_HIP(launch_fill2_u32(plan->d_queues, nq, reinterpret_cast<uint32_t*>(counters), 2 * n_counters, 0, s));
    if (clear_bits && bits)
        PC_HIP(launch_clear_ranges(bits, plan->d_clear, (uint32_t)(plan->clear.size() / 2), s));
    const int want = strategy == 2 ? 2 : strategy == 3 ? 1 : kBranches;
    const int nb = (int)std::min<size_t>(want, plan->batched.size());
    // work independent of the buckets (after the fills) goes first onto a
    // branch of its own when one is free, else onto the last one
    const int ns = side ? std::min(kBranches, std::max(nb, 1) + 1) : nb;
    PC_HIP(fork_branches(ws, s, ns));
    if (side) PC_HIP(side(branch_stream(ws, s, ns - 1)));
    auto lds_class = [](const Bucket& bk) { return bk.cls == kAMap || bk.cls == kALds; };
    auto weight = [&](const Bucket& bk) { return (strategy == 1 && lds_class(bk)) ? 3.0 * bk.cost : bk.cost; };
    std::vector<size_t> idx(plan->batched.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](size_t x, size_t y) {
        const Bucket &bx = plan->batched[x], &by = plan->batched[y];
        if (strategy == 4 && lds_class(bx) != lds_class(by)) return lds_class(bx);
        return weight(bx) > weight(by);
    });
    std::vector<double> load(nb > 1 ? nb : 1, 0.0);
    int next_own = 0;
    for (size_t qi : idx) {
        const Bucket& bk = plan->batched[qi];
        int br = 0;
        if (strategy == 4 && lds_class(bk) && next_own < (int)load.size()) {
            br = next_own++;
        } else {
            for (int b = 1; b < (int)load.size(); ++b)
                if (load[b] < load[br]) br = b;
        }
        load[br] += weight(bk);
        hipStream_t bs = branch_stream(ws, s, br);
        SweepArgs a;
        a.tasks = plan->d_lpt + bk.first;
        a.n_tasks = bk.count;
        a.persistent = 1;
        a.queue = plan->d_queues + qi;
        a.jobs = plan->d_jobs;
        a.models = plan->d_models;
        a.probes = plan->d_probes;
        a.counters = counters;
        a.bits = bits;
        a.zeros = plan->zeros;
        a.abort_flag = abort_flag_dev();
        a.aborted = plan->d_queues + plan->batched.size();
        a.lds_rows = bk.lds_rows;
        a.map_rows = bk.map_rows;
        a.bm_words = bk.bm_words;
        int occ = 0;
        PC_HIP(sweep_occupancy(score, bk.pol, bk.cls, bk.lds_rows, bk.bm_words, &occ));
        uint32_t blocks = (uint32_t)std::max(occ, 1) * (uint32_t)ws->cus;
        uint32_t threads;
        size_t lds;
        sweep_geometry(bk.cls, bk.lds_rows, bk.bm_words, &threads, &lds);
        const uint32_t wpb = threads / kWave;
        const uint32_t need = (bk.count + wpb - 1) / wpb;
        if (need < blocks) blocks = need;
        PC_HIP(launch_sweep(score, bk.pol, bk.cls, a, blocks, bs));
    }
    PC_HIP(join_branches(ws, s, ns));
    if (tail) PC_HIP(tail(s));
    return PCHASE_OK;
}

int run_sweep_plan(Workspace* ws, SweepPlan* plan, bool score, uint64_t* counters, uint64_t n_counters,
                   uint32_t* bits, bool clear_bits, uint32_t mode, hipStream_t stream,
                   const std::function<hipError_t(hipStream_t)>& tail, bool autotune, bool defer_tuning,
                   const std::function<hipError_t(hipStream_t)>& side) {
    if (mode == PCHASE_PLAIN) {
        const uint32_t nq = (uint32_t)plan->batched.size() + 2;
        PC_HIP(launch_fill2_u32(plan->d_queues, nq, reinterpret_cast<uint32_t*>(counters), 2 * n_counters, 0, stream));
        if (clear_bits && bits)
            PC_HIP(launch_clear_ranges(bits, plan->d_clear, (uint32_t)(plan->clear.size() / 2), stream));
        if (side) PC_HIP(side(stream));
        for (const Bucket& bk : plan->plain) {
            if (bk.count == 0) continue;
            SweepArgs a;
            a.tasks = plan->d_plain + bk.first;
            a.n_tasks = bk.count;
            a.persistent = 0;
            a.queue = nullptr;
            a.jobs = plan->d_jobs;
            a.models = plan->d_models;
            a.probes = plan->d_probes;
            a.counters = counters;
            a.bits = bits;
            a.zeros = plan->zeros;
            a.abort_flag = nullptr;
            a.aborted = nullptr;
            a.lds_rows = bk.lds_rows;
            a.map_rows = bk.map_rows;
            a.bm_words = bk.bm_words;
            uint32_t threads;
            size_t lds;
            sweep_geometry(bk.cls, bk.lds_rows, bk.bm_words, &threads, &lds);
            const uint32_t wpb = threads / kWave;
            PC_HIP(launch_sweep(score, bk.pol, bk.cls, a, (bk.count + wpb - 1) / wpb, stream));
        }
        if (tail) PC_HIP(tail(stream));
        return PCHASE_OK;
    }

    // a flag already set when the run starts stops it before anything is
    // launched (the persistent kernels only poll it every 64th pull)
    if (abort_flag_host() != 0) return set_error(PCHASE_EABORTED, "replay aborted by pchase_abort");
    // batched: the sequence is launched directly on every run (about twenty
    // launches against milliseconds of kernel time).  With autotune, a run
    // of a plan that has not been tuned yet times every branch strategy on
    // the stream and keeps the fastest for the later runs; the last timed
    // run uses the chosen strategy, so its outputs are this run's.  With
    // defer_tuning the run uses the current strategy and leaves the tuning
    // to the next one (a problem's first answer does not wait for it).
    const bool tunable = autotune && plan->batched.size() >= 2 && !plan->tuned;
    if (!tunable || defer_tuning)
        return enqueue_batched(ws, plan, score, counters, n_counters, bits, clear_bits, stream, tail, side,
                               plan->strategy);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipError_t e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    int best = 0;
    float best_ms = 0;
    int rc = PCHASE_OK;
    for (int st = 0; st < kStrategies && e == hipSuccess && rc == PCHASE_OK; ++st) {
        float ms = 0;
        for (int r = 0; r < 2 && e == hipSuccess && rc == PCHASE_OK; ++r) {   // the first run warms up
            e = hipEventRecord(t0, stream);
            if (e == hipSuccess)
                rc = enqueue_batched(ws, plan, score, counters, n_counters, bits, clear_bits, stream, tail, side, st);
            if (e == hipSuccess && rc == PCHASE_OK) e = hipEventRecord(t1, stream);
            if (e == hipSuccess && rc == PCHASE_OK) e = hipEventSynchronize(t1);
            if (e == hipSuccess && rc == PCHASE_OK) e = hipEventElapsedTime(&ms, t0, t1);
        }
        if (e == hipSuccess && rc == PCHASE_OK && (st == 0 || ms < best_ms)) {
            best = st;
            best_ms = ms;
        }
    }
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    if (rc) return rc;
    if (e != hipSuccess) return hip_fail(e, "autotune run");
    // timings of replays that pchase_abort cut short say nothing: the plan
    // stays untuned and the next run tunes again
    if (abort_flag_host() == 0) {
        plan->strategy = best;
        plan->tuned = true;
    }
    return enqueue_batched(ws, plan, score, counters, n_counters, bits, clear_bits, stream, tail, side,
                           plan->strategy);
}

}  // namespace pc
