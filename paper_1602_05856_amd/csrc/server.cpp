// Serving loop: graph-build jobs submitted at any time, run by worker
// threads that each own a stream and a reusable plan.
//
//   admission   twice per job.  First its first-pass bytes (input, filter,
//               bitmaps, layout tables) are estimated from its size; a worker
//               starts the oldest queued job only when the bytes every worker
//               holds or has reserved, plus this one, fit the HBM budget
//               (idle workers give their cached buffers back when needed);
//               jobs wait in arrival order, so a large job is never starved.
//               Then, once the first pass has counted the candidates, the run
//               reserves its exact table and later its outputs the same way
//               (the grow hook), waiting for other jobs when they do not fit
//               yet; so the bytes all workers hold never exceed the budget
//   lanes       express workers take only small jobs; when CUs are kept for
//               them, they alone take small jobs, whose kernels then never
//               queue for CUs behind a large job's persistent grids
//   batching    a worker that takes a small job also takes the queued small
//               jobs behind it that share k, h and flags, and runs them as
//               one batched plan (every phase one launch over all of them)
//   reuse       a worker's plan and input buffer keep their device memory
//               from job to job and only grow, so a warm server allocates no
//               device memory
//   overlap     workers run on their own streams, so one job's passes run
//               beside another's
//
// A job's outputs do not depend on what it was batched or overlapped with:
// every set of a batch has its own filter, table, sentinels and outputs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hostmem.hpp"
#include "runtime.hpp"

using namespace tp;

namespace {

using Clock = std::chrono::steady_clock;

struct Job {
    uint64_t id = 0;
    uint32_t k = 0, h = 0, flags = 0;
    uint64_t b = 0;
    std::vector<void *> blocks;      // page-locked copies of the genomes
    std::vector<tp_genome> genomes;  // point into blocks
    uint64_t bases = 0, est_bytes = 0;
    tp_job_info info{};
    bool done = false;
    bool claimed = false;  // a caller is blocked in tp_server_wait for it
    int rc = TP_OK;
    std::string err;
    tp_result *result = nullptr;

    Job() = default;
    Job(const Job &) = delete;
    Job &operator=(const Job &) = delete;
    ~Job() {
        for (void *b : blocks)
            host_free(b);
    }
};

// Device bytes a job needs before its first pass ends (the first admission
// point): the input laid out in tiles, the filter, the binned fill's
// scratch (large filters), the candidate and junction bitmaps, and the
// layout tables, counters and sentinel tables
// (bounded by a few bytes per base plus a fixed margin).  The exact table and
// the outputs depend on the data: the run asks for them at the second
// admission point (the grow hook), when the first pass has counted the
// candidates.
uint64_t estimate_bytes(uint64_t bases, uint32_t n_genomes, uint64_t b, uint32_t k) {
    const uint64_t W = k <= 31 ? 1 : (k <= 63 ? 2 : 4);
    const uint64_t laid = bases + (uint64_t)n_genomes * TILE + TILE;  // tile-aligned positions
    const uint64_t tiles = laid / TILE + 1;
    // a filter of 1 GiB or more is filled binned (the default), with 16
    // bytes of scratch per position of a chunk of at most 2^31
    const uint64_t bin = b / 8 >= (1ull << 30) ? 16 * std::min<uint64_t>(laid, 1ull << 31) : 0;
    return laid / 4 + b / 8 + 3 * (laid / 8) + tiles * (4 + sizeof(TileInfo)) +
           (uint64_t)n_genomes * 16 * (8 * W + 4) + bin + (64ull << 20);
}

}  // namespace

struct tp_server {
    tp_server_opts o{};
    int device = 0;
    Clock::time_point t0;
    std::mutex m;
    std::condition_variable cv_work, cv_done;
    std::deque<Job *> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs;
    uint64_t next_id = 1;
    bool stop = false;
    bool reclaim = false;  // an admission is waiting for idle workers' buffers
    uint32_t waiters = 0;  // callers blocked in tp_server_wait
    tp_server_stats st{};

    struct Worker {
        std::thread th;
        hipStream_t stream = nullptr;
        tp_plan *plan = nullptr;
        DevBuf input;
        uint64_t held = 0;      // device bytes its plan and input hold
        uint64_t reserved = 0;  // estimate of the group it is running
        bool busy = false;
        bool growing = false;   // waiting at the second admission point
        uint32_t index = 0;
        tp_server *srv = nullptr;
    };
    std::vector<std::unique_ptr<Worker>> workers;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

    uint64_t held_by_others(const Worker *me) const {
        uint64_t n = 0;
        for (const auto &w : workers)
            if (w.get() != me)
                n += w->busy ? std::max(w->held, w->reserved) : w->held;
        return n;
    }

    void update_totals() {
        uint64_t n = 0;
        for (const auto &w : workers)
            n += w->held;
        st.held_bytes = n;
        st.peak_held_bytes = std::max(st.peak_held_bytes, n);
    }

    void worker_loop(Worker *w);
    void run_group(Worker *w, std::vector<Job *> &group);
    int grow(Worker *w, uint64_t plan_bytes);
};

// The second admission point: a running job's plan is about to grow to
// plan_bytes (its exact table, or its outputs).  The worker's reservation
// grows with it when everything fits the budget; otherwise it waits for other
// jobs to finish (or idle workers to hand back their buffers), and fails
// with TP_ENOMEM when nothing that could free memory is left.
int tp_server::grow(Worker *w, uint64_t plan_bytes) {
    std::unique_lock<std::mutex> lk(m);
    const uint64_t need = plan_bytes + w->input.cap;
    for (;;) {
        if (need <= w->reserved)
            return TP_OK;
        if (held_by_others(w) + need <= o.hbm_budget) {
            w->reserved = need;
            return TP_OK;
        }
        bool idle_cache = false, running = false;
        for (const auto &v : workers) {
            if (v.get() == w)
                continue;
            idle_cache |= !v->busy && v->held;
            running |= v->busy && !v->growing;
        }
        if (!idle_cache && !running)
            return fail(TP_ENOMEM, "job needs " + std::to_string(need) +
                                       " device bytes; the server budget is " +
                                       std::to_string(o.hbm_budget) + " and nothing else runs");
        reclaim = idle_cache;
        if (reclaim)
            cv_work.notify_all();
        w->growing = true;
        cv_work.wait(lk);
        w->growing = false;
    }
}

static int server_grow_hook(void *ctx, uint64_t bytes) {
    auto *w = (tp_server::Worker *)ctx;
    return w->srv->grow(w, bytes);
}

void tp_server::run_group(Worker *w, std::vector<Job *> &group) {
    std::vector<tp_set> sets(group.size());
    for (size_t i = 0; i < group.size(); ++i) {
        sets[i].genomes = group[i]->genomes.data();
        sets[i].n_genomes = (uint32_t)group[i]->genomes.size();
        sets[i].reserved = 0;
        sets[i].bloom_bits = group[i]->b;
    }
    const Job &j0 = *group[0];
    auto ms_since = [](Clock::time_point t) {
        return std::chrono::duration<float, std::milli>(Clock::now() - t).count();
    };
    auto t = Clock::now();
    int rc = plan_layout(w->plan, sets.data(), (uint32_t)sets.size(), j0.k, j0.h, j0.flags);
    if (!rc && (o.wg_per_cu || o.table_budget_mib)) {
        tp_config c = w->plan->cfg;
        if (o.wg_per_cu)
            for (auto &x : c.wg_per_cu)
                x = o.wg_per_cu;
        c.table_budget = (uint64_t)o.table_budget_mib << 20;
        rc = tp_plan_set_config(w->plan, &c);
    }
    const float layout_ms = ms_since(t);
    t = Clock::now();
    if (!rc) {
        const hipError_t e = w->input.ensure(std::max<uint64_t>(w->plan->input_bytes, 16));
        if (e != hipSuccess)
            rc = fail(e == hipErrorOutOfMemory ? TP_ENOMEM : TP_EDEVICE,
                      std::string("input buffer: ") + hipGetErrorString(e));
    }
    if (!rc)
        rc = tp_batch_upload(w->plan, sets.data(), w->input.as<uint8_t>(), w->stream);
    if (!rc) {
        const hipError_t e = hipStreamSynchronize(w->stream);
        if (e != hipSuccess)
            rc = fail(TP_EDEVICE, std::string("upload: ") + hipGetErrorString(e));
    }
    const float upload_ms = ms_since(t);
    t = Clock::now();
    if (!rc)
        rc = tp_run(w->plan, w->input.as<uint8_t>(), w->stream);
    const float run_ms = ms_since(t);
    for (size_t i = 0; i < group.size(); ++i) {
        Job &j = *group[i];
        t = Clock::now();
        j.rc = rc ? rc : tp_download_set(w->plan, (uint32_t)i, w->stream, &j.result);
        if (j.rc)
            j.err = twopaco_last_error();
        j.info.layout_ms = layout_ms;
        j.info.upload_ms = upload_ms;
        j.info.run_ms = run_ms;
        j.info.download_ms = ms_since(t);
    }
}

void tp_server::worker_loop(Worker *w) {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(m);
    for (;;) {
        if (stop)
            break;
        if (reclaim && !w->busy && w->held) {
            // give cached buffers back for a waiting admission
            plan_release(w->plan);
            w->input.release();
            w->held = 0;
            update_totals();
            cv_work.notify_all();
        }
        if (queue.empty()) {
            cv_work.wait(lk);
            continue;
        }
        // the oldest job (an express worker: the oldest small job; with CUs
        // kept for the express workers, another worker: the oldest job that
        // is not small), plus the small compatible jobs queued behind it
        size_t first = 0;
        const bool express = w->index + o.express_workers >= o.workers;
        const bool skip_small = !express && o.express_cus;
        while (first < queue.size() && (express ? queue[first]->bases > o.batch_max_bases
                                                : skip_small &&
                                                      queue[first]->bases <= o.batch_max_bases))
            ++first;
        if (first == queue.size()) {
            cv_work.wait(lk);
            continue;
        }
        std::vector<Job *> group{queue[first]};
        uint64_t est = queue[first]->est_bytes, bases = queue[first]->bases;
        const Job &j0 = *queue[first];
        if (o.max_batch > 1 && j0.bases <= o.batch_max_bases) {
            for (size_t i = first + 1; i < queue.size() && group.size() < o.max_batch; ++i) {
                const Job &j = *queue[i];
                if (j.k != j0.k || j.h != j0.h || j.flags != j0.flags ||
                    j.bases > o.batch_max_bases || bases + j.bases > o.batch_total_bases)
                    continue;
                group.push_back(queue[i]);
                est += j.est_bytes;
                bases += j.bases;
            }
        }
        const uint64_t others = held_by_others(w);
        if (others + std::max(w->held, est) > o.hbm_budget) {
            while (group.size() > 1) {  // try the first job alone
                est -= group.back()->est_bytes;
                group.pop_back();
            }
            if (others + std::max(w->held, est) > o.hbm_budget) {
                bool idle_cache = false;
                for (const auto &v : workers)
                    idle_cache |= v.get() != w && !v->busy && v->held;
                bool anyone_busy = false;
                for (const auto &v : workers)
                    anyone_busy |= v->busy;
                if (!idle_cache && !anyone_busy && w->held > est) {
                    // this worker's own cache is what is in the way
                    plan_release(w->plan);
                    w->input.release();
                    w->held = 0;
                    update_totals();
                    continue;
                }
                if (!idle_cache && !anyone_busy) {
                    // nothing will ever free enough memory: the job cannot run
                    Job *j = queue[first];
                    queue.erase(queue.begin() + (std::ptrdiff_t)first);
                    j->rc = TP_ENOMEM;
                    j->err = "job needs about " + std::to_string(j->est_bytes) +
                             " device bytes; the server budget is " +
                             std::to_string(o.hbm_budget);
                    j->done = true;
                    ++st.failed;
                    ++st.completed;
                    cv_done.notify_all();
                    continue;
                }
                reclaim = idle_cache;
                if (reclaim)
                    cv_work.notify_all();
                cv_work.wait(lk);
                continue;
            }
        }
        reclaim = false;
        for (Job *j : group)
            queue.erase(std::find(queue.begin(), queue.end(), j));
        w->busy = true;
        w->reserved = est;
        const double t = now();
        for (Job *j : group) {
            j->info.start_s = t;
            j->info.batch_jobs = (uint32_t)group.size();
            j->info.worker = w->index;
        }
        ++st.batches;
        st.running += group.size();
        st.queued = queue.size();
        lk.unlock();
        run_group(w, group);
        const uint64_t held = plan_device_bytes(w->plan) + w->input.cap;
        lk.lock();
        const double t1 = now();
        for (Job *j : group) {
            j->info.end_s = t1;
            j->done = true;
            ++st.completed;
            st.failed += j->rc != TP_OK;
        }
        st.running -= group.size();
        w->busy = false;
        w->reserved = 0;
        w->held = held;
        update_totals();
        cv_done.notify_all();
        cv_work.notify_all();
    }
}

extern "C" int tp_server_create(const tp_server_opts *opts, tp_server **out) {
    if (!out)
        return fail(TP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!opts)
        return fail(TP_EINVAL, "opts is NULL");
    if (opts->workers < 1 || opts->workers > 16)
        return fail(TP_EINVAL, "workers must be in 1..16");
    if (opts->express_workers >= opts->workers)
        return fail(TP_EINVAL, "express_workers must be < workers");
    if (opts->max_batch < 1)
        return fail(TP_EINVAL, "max_batch must be >= 1");
    if (opts->hbm_budget == 0)
        return fail(TP_EINVAL, "hbm_budget must be > 0");
    if (opts->wg_per_cu > 64)
        return fail(TP_EINVAL, "wg_per_cu must be 0 (all that fit) or 1..64");
    if (opts->express_cus && !opts->express_workers)
        return fail(TP_EINVAL, "express_cus needs express_workers");
    std::unique_ptr<tp_server> s(new (std::nothrow) tp_server);
    if (!s)
        return fail(TP_ENOMEM, "host allocation failed");
    s->o = *opts;
    s->t0 = Clock::now();
    HIPCHK(hipGetDevice(&s->device));
    int ncu = 0;
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, s->device));
    if (opts->express_cus >= (uint32_t)ncu)
        return fail(TP_EINVAL, "express_cus must leave CUs for the other workers");
    // CU masks: the first express_cus CUs for express workers, the rest for
    // the others
    const uint32_t mask_words = ((uint32_t)ncu + 31) / 32;
    std::vector<uint32_t> m_express(mask_words, 0), m_other(mask_words, 0);
    for (uint32_t cu = 0; cu < (uint32_t)ncu; ++cu)
        (cu < opts->express_cus ? m_express : m_other)[cu / 32] |= 1u << (cu % 32);
    for (uint32_t i = 0; i < opts->workers; ++i) {
        auto w = std::make_unique<tp_server::Worker>();
        w->index = i;
        const bool express = i + opts->express_workers >= opts->workers;
        if (opts->express_cus) {
            const std::vector<uint32_t> &mk = express ? m_express : m_other;
            HIPCHK(hipExtStreamCreateWithCUMask(&w->stream, mask_words, mk.data()));
        } else {
            HIPCHK(hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking));
        }
        w->plan = new (std::nothrow) tp_plan;
        if (!w->plan) {
            (void)hipStreamDestroy(w->stream);
            return fail(TP_ENOMEM, "host allocation failed");
        }
        w->srv = s.get();
        w->plan->grow_hook = server_grow_hook;
        w->plan->grow_ctx = w.get();
        if (opts->express_cus)
            w->plan->cu_limit = express ? opts->express_cus : (uint32_t)ncu - opts->express_cus;
        s->workers.push_back(std::move(w));
    }
    tp_server *raw = s.get();
    for (auto &w : s->workers) {
        tp_server::Worker *wp = w.get();
        w->th = std::thread([raw, wp] { raw->worker_loop(wp); });
    }
    *out = s.release();
    return TP_OK;
}

extern "C" int tp_server_submit(tp_server *s, const tp_genome *genomes, uint32_t n_genomes,
                                uint32_t k, uint64_t bloom_bits, uint32_t hash_count,
                                uint32_t flags, uint64_t *job_id) {
    if (!s || !job_id)
        return fail(TP_EINVAL, "NULL argument");
    // validate as a plan would (host work only)
    tp_plan *probe = nullptr;
    int rc = tp_plan_create(genomes, n_genomes, k, bloom_bits, hash_count, flags, &probe);
    if (rc)
        return rc;
    tp_plan_destroy(probe);
    auto j = std::make_unique<Job>();
    j->k = k;
    j->h = hash_count;
    j->flags = flags;
    j->b = bloom_bits;
    // one page-locked block per job: all packed genomes, then all N runs
    uint64_t bytes = 0, run_words = 0;
    for (uint32_t g = 0; g < n_genomes; ++g) {
        bytes += align_up((genomes[g].n_bases + 3) / 4, 64);
        run_words += 2 * genomes[g].n_nruns;
    }
    uint8_t *blk = (uint8_t *)host_alloc(bytes + run_words * 8 + 64);
    if (!blk)
        return fail(TP_ENOMEM, "host allocation failed");
    j->blocks.push_back(blk);
    uint8_t *cur = blk;
    uint64_t *runs = (uint64_t *)(blk + align_up(bytes, 64));
    j->genomes.resize(n_genomes);
    for (uint32_t g = 0; g < n_genomes; ++g) {
        const tp_genome &G = genomes[g];
        const uint64_t nbytes = (G.n_bases + 3) / 4;
        tp_genome &C = j->genomes[g];
        C.packed = nullptr;
        C.n_runs = nullptr;
        if (nbytes && G.packed) {
            std::memcpy(cur, G.packed, nbytes);
            C.packed = cur;
        }
        cur += align_up(nbytes, 64);
        if (G.n_nruns) {
            std::memcpy(runs, G.n_runs, G.n_nruns * 16);
            C.n_runs = runs;
            runs += 2 * G.n_nruns;
        }
        C.n_bases = G.n_bases;
        C.n_nruns = G.n_nruns;
        j->bases += G.n_bases;
    }
    // a set sized by the plan (bloom_bits 0) gets at most 32 bits per base
    // (a power of two at 16 bits per (k+1)-mer)
    j->est_bytes = estimate_bytes(j->bases, n_genomes, bloom_bits ? bloom_bits : 32 * j->bases, k);
    std::lock_guard<std::mutex> lk(s->m);
    if (s->stop)
        return fail(TP_ESTATE, "server is stopping");
    j->id = s->next_id++;
    j->info.submit_s = s->now();
    j->info.bases = j->bases;
    *job_id = j->id;
    s->queue.push_back(j.get());
    s->jobs[j->id] = std::move(j);
    ++s->st.submitted;
    s->st.queued = s->queue.size();
    s->cv_work.notify_all();  // an express worker may not take this job
    return TP_OK;
}

// Wait for (or with poll, look at) a job.  One caller at a time may wait for
// a job; it is forgotten once its result is handed out.
static int wait_or_poll(tp_server *s, uint64_t job_id, int64_t timeout_ms, bool poll,
                        tp_result **out, tp_job_info *info) {
    if (!s || !out)
        return fail(TP_EINVAL, "NULL argument");
    *out = nullptr;
    std::unique_lock<std::mutex> lk(s->m);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end())
        return fail(TP_EINVAL, "unknown job " + std::to_string(job_id));
    Job *j = it->second.get();
    if (j->claimed)
        return fail(TP_ESTATE, "job " + std::to_string(job_id) + " is waited for by another caller");
    if (!j->done) {
        if (poll || s->stop)
            return poll && !s->stop
                       ? fail(TP_EPENDING, "job " + std::to_string(job_id) + " has not finished")
                       : fail(TP_ESTATE, "server is stopping");
        j->claimed = true;
        ++s->waiters;
        auto ready = [&] { return j->done || s->stop; };
        if (timeout_ms < 0)
            s->cv_done.wait(lk, ready);
        else
            (void)s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
        j->claimed = false;
        --s->waiters;
        if (s->stop)
            s->cv_done.notify_all();  // tp_server_destroy waits for the waiters to leave
        if (!j->done)
            return s->stop ? fail(TP_ESTATE, "server is stopping")
                           : fail(TP_ETIMEOUT, "job " + std::to_string(job_id) + " still running");
        it = s->jobs.find(job_id);  // still there: only a caller that claimed it erases it
    }
    if (info)
        *info = j->info;
    const int rc = j->rc;
    const std::string err = j->err;
    *out = j->result;
    j->result = nullptr;
    s->jobs.erase(it);
    return rc ? fail(rc, err) : TP_OK;
}

extern "C" int tp_server_wait(tp_server *s, uint64_t job_id, int64_t timeout_ms, tp_result **out,
                              tp_job_info *info) {
    return wait_or_poll(s, job_id, timeout_ms, false, out, info);
}

extern "C" int tp_server_poll(tp_server *s, uint64_t job_id, tp_result **out, tp_job_info *info) {
    return wait_or_poll(s, job_id, 0, true, out, info);
}

extern "C" int tp_server_get_stats(tp_server *s, tp_server_stats *out) {
    if (!s || !out)
        return fail(TP_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->m);
    *out = s->st;
    out->queued = s->queue.size();
    return TP_OK;
}

extern "C" void tp_server_destroy(tp_server *s) {
    if (!s)
        return;
    {
        std::lock_guard<std::mutex> lk(s->m);
        s->stop = true;
        for (Job *j : s->queue) {
            j->rc = TP_ESTATE;
            j->err = "server stopped before the job ran";
            j->done = true;
        }
        s->queue.clear();
        s->cv_work.notify_all();
        s->cv_done.notify_all();
    }
    {
        // callers blocked in tp_server_wait wake (stop) and leave first
        std::unique_lock<std::mutex> lk(s->m);
        s->cv_done.wait(lk, [&] { return s->waiters == 0; });
    }
    for (auto &w : s->workers)
        if (w->th.joinable())
            w->th.join();
    for (auto &w : s->workers) {
        tp_plan_destroy(w->plan);
        w->input.release();
        if (w->stream)
            (void)hipStreamDestroy(w->stream);
    }
    for (auto &kv : s->jobs)
        twopaco_result_free(kv.second->result);
    delete s;
}
