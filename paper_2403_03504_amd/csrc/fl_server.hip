// Layout server: continuous batching of layout jobs on one GPU.
//
// Jobs (a directed edge list, initial positions, ForceAtlas2 parameters and
// an iteration count, all in host memory) are copied at submission and queued
// first-in first-out.  `slots` worker threads each own a HIP stream and an
// fl_ctx; a free worker admits the job at the head of the queue as soon as the
// estimated device bytes of the jobs running plus its own fit the budget (the
// head is never overtaken, so no job starves).  A running job stays on the
// device from upload to result: CSR build, components, Kamada-Kawai /
// ForceAtlas2 layout (fl_layout), download.  Jobs on different workers run
// concurrently on their own streams; each job's kernels see only its own
// data and reduce in a fixed order, so a result does not depend on what else
// is running.
//
// A host-only executor (fake_ns_per_update > 0) sleeps instead of launching
// kernels, so the admission policy can be tested without a GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "fl_common.h"

namespace {

struct Job {
    uint64_t id = 0;
    int32_t n = 0;
    int64_t m = 0;
    std::vector<int32_t> src, dst;
    std::vector<float> x, y;
    int32_t iters = 0;
    fl_fa2_params prm{};
    fl_tuning tuning{};  // the server's table when the job was admitted
    int32_t state = FL_JOB_QUEUED;
    double t_arrive = 0, t_start = 0, t_done = 0;
    size_t bytes = 0;
    std::string err;
    bool cancel = false;
};

// Device bytes a job may hold: CSR build (sort keys), graph, positions and
// the FMM workspace (tree, lists, expansions; about 700 B per node at the
// default leaf size).
size_t job_bytes(int64_t n, int64_t m) { return (size_t)(700 * n + 48 * m + (16 << 20)); }

}  // namespace

struct fl_server {
    int device = 0;
    size_t budget = 0;
    int slots = 1;
    double fake_ns = 0.0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Job>> queue;
    std::map<uint64_t, std::shared_ptr<Job>> jobs;
    size_t in_use = 0, peak = 0;  // sum of the workers' charges (below)
    // per worker: device bytes held while idle (context workspace, branch
    // contexts, job buffers), and its charge against the budget: the held
    // bytes when idle, max(held, the job's estimate) while a job runs
    std::vector<size_t> held, charge;
    std::vector<char> busy;
    size_t peak_held = 0;
    uint64_t next_id = 1;
    bool stop = false;
    std::vector<std::thread> workers;
    std::chrono::steady_clock::time_point origin = std::chrono::steady_clock::now();
    fl_server_stats st{};
    fl_tuning tuning{};
    std::string err;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - origin).count();
    }
};

namespace {

struct DevArrays {
    int32_t *src = nullptr, *dst = nullptr, *rp = nullptr, *col = nullptr, *deg = nullptr;
    float *x = nullptr, *y = nullptr;
    int64_t cap_n = 0, cap_m = 0;
    size_t bytes() const { return cap_n ? (size_t)(4 * (cap_n + 1) + 12 * cap_n + 16 * cap_m) : 0; }
    void release_held()  // with AllocGuard held
    {
        for (void *p : {(void *)src, (void *)dst, (void *)rp, (void *)col, (void *)deg, (void *)x, (void *)y})
            if (p) (void)hipFree(p);
        *this = DevArrays{};
    }
    void release()
    {
        fl::AllocGuard guard;
        release_held();
    }
    bool ensure(int64_t n, int64_t m)
    {
        if (n <= cap_n && m <= cap_m) return true;
        fl::AllocGuard guard;
        release_held();
        const int64_t nn = std::max<int64_t>(n, 1), mm = std::max<int64_t>(m, 1);
        bool ok = hipMalloc(&src, 4 * mm) == hipSuccess && hipMalloc(&dst, 4 * mm) == hipSuccess &&
                  hipMalloc(&rp, 4 * (nn + 1)) == hipSuccess && hipMalloc(&col, 8 * mm) == hipSuccess &&
                  hipMalloc(&deg, 4 * nn) == hipSuccess && hipMalloc(&x, 4 * nn) == hipSuccess &&
                  hipMalloc(&y, 4 * nn) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            release_held();
            return false;
        }
        cap_n = nn;
        cap_m = mm;
        return true;
    }
};

void run_on_gpu(fl_ctx *ctx, hipStream_t s, DevArrays &d, Job &j)
{
    if (!d.ensure(j.n, j.m)) throw fl::Error(FL_ENOMEM, "job buffers do not fit on the device");
    if (j.m > 0) {
        FL_CHECK_HIP(hipMemcpyAsync(d.src, j.src.data(), 4 * j.m, hipMemcpyHostToDevice, s));
        FL_CHECK_HIP(hipMemcpyAsync(d.dst, j.dst.data(), 4 * j.m, hipMemcpyHostToDevice, s));
    }
    FL_CHECK_HIP(hipMemcpyAsync(d.x, j.x.data(), 4 * (size_t)j.n, hipMemcpyHostToDevice, s));
    FL_CHECK_HIP(hipMemcpyAsync(d.y, j.y.data(), 4 * (size_t)j.n, hipMemcpyHostToDevice, s));
    int64_t nnz = 0;
    fl_status rc = fl_set_tuning(ctx, &j.tuning);
    if (rc != FL_OK) throw fl::Error(rc, fl_last_error(ctx));
    rc = fl_build_csr(ctx, j.n, j.m, d.src, d.dst, d.rp, d.col, d.deg, &nnz);
    if (rc != FL_OK) throw fl::Error(rc, fl_last_error(ctx));
    fl_kk_params kk;
    fl_kk_default_params(&kk);
    rc = fl_layout(ctx, j.n, d.rp, d.col, d.deg, d.x, d.y, &j.prm, j.iters, &kk, 256, 4096, nullptr);
    if (rc != FL_OK) throw fl::Error(rc, fl_last_error(ctx));
    FL_CHECK_HIP(hipMemcpyAsync(j.x.data(), d.x, 4 * (size_t)j.n, hipMemcpyDeviceToHost, s));
    FL_CHECK_HIP(hipMemcpyAsync(j.y.data(), d.y, 4 * (size_t)j.n, hipMemcpyDeviceToHost, s));
    FL_CHECK_HIP(hipStreamSynchronize(s));
    // a quiet point: free the workspace the job's growth retired (the
    // branch contexts of its batches keep theirs until they grow or end)
    fl::free_retired(ctx);
    for (auto *sc : ctx->sub) fl::free_retired(sc);
}

// Device bytes a worker holds between jobs: its context's workspace (with
// the branch contexts') and its job buffers.
size_t worker_held(const fl_ctx *ctx, const DevArrays &d)
{
    size_t b = d.bytes();
    if (ctx) {
        b += fl_workspace_bytes(ctx);
        for (auto *sc : ctx->sub) b += fl_workspace_bytes(sc);
    }
    return b;
}

// Give back everything a worker holds (a fresh context on the same stream).
bool worker_trim(fl_server *sv, fl_ctx *&ctx, hipStream_t s, DevArrays &d)
{
    d.release();
    if (!ctx) return true;
    fl_destroy(ctx);
    ctx = nullptr;
    if (fl_create(&ctx, sv->device, s, 0) != FL_OK) return false;
    // the workers capture concurrently; their iterations keep every launch
    // on the job's own streams (no branch streams, see below)
    ctx->branches = false;
    return true;
}

size_t total_charge(const fl_server *sv)
{
    size_t t = 0;
    for (size_t c : sv->charge) t += c;
    return t;
}

size_t running_charge(const fl_server *sv)
{
    size_t t = 0;
    for (size_t w = 0; w < sv->charge.size(); ++w)
        if (sv->busy[w]) t += sv->charge[w];
    return t;
}

void worker(fl_server *sv, int me)
{
    hipStream_t s = nullptr;
    fl_ctx *ctx = nullptr;
    DevArrays d;
    std::string init_err;
    if (sv->fake_ns <= 0.0) {
        if (hipSetDevice(sv->device) != hipSuccess || hipStreamCreate(&s) != hipSuccess ||
            fl_create(&ctx, sv->device, s, 0) != FL_OK)
            init_err = "worker could not create its stream/context";
        // the workers capture concurrently; their iterations keep every
        // launch on the job's own streams (no branch streams): a run with
        // branch streams inside concurrent captures ended in a host crash
        // whose cause is not established
        if (ctx) ctx->branches = false;
    }
    while (true) {
        std::shared_ptr<Job> j;
        bool trim = false;
        size_t held_before = 0;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_work.wait(lk, [&] {
                if (sv->stop) return true;
                if (sv->queue.empty()) return false;
                const size_t b = sv->queue.front()->bytes;
                const size_t mine = std::max(sv->held[me], b);
                if (total_charge(sv) - sv->charge[me] + mine <= sv->budget) return true;
                // the head does not fit, but would without the memory idle
                // workers hold: this idle worker gives its memory back
                if (sv->held[me] > 0 && running_charge(sv) + b <= sv->budget) {
                    trim = true;
                    return true;
                }
                return false;
            });
            if (sv->stop) break;
            if (!trim) {
                j = sv->queue.front();
                sv->queue.pop_front();
                j->state = FL_JOB_RUNNING;
                j->t_start = sv->now();
                j->tuning = sv->tuning;
                sv->busy[me] = 1;
                held_before = sv->held[me];
                sv->charge[me] = std::max(sv->held[me], j->bytes);
                sv->in_use = total_charge(sv);
                sv->peak = std::max(sv->peak, sv->in_use);
                sv->st.admitted++;
            }
        }
        if (trim) {
            if (sv->fake_ns <= 0.0 && !worker_trim(sv, ctx, s, d) && init_err.empty())
                init_err = "worker could not recreate its context";
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->held[me] = sv->charge[me] = worker_held(ctx, d);
            sv->in_use = total_charge(sv);
            sv->st.trims++;
            sv->cv_work.notify_all();
            continue;
        }
        std::string jerr;
        fl_status jrc = FL_OK;
        try {
            if (!init_err.empty()) throw fl::Error(FL_EHIP, init_err);
            if (sv->fake_ns > 0.0) {
                const double secs = sv->fake_ns * 1e-9 * (double)j->n * (double)std::max(j->iters, 1);
                std::this_thread::sleep_for(std::chrono::duration<double>(secs));
            } else {
                FL_CHECK_HIP(hipSetDevice(sv->device));
                run_on_gpu(ctx, s, d, *j);
            }
        } catch (const fl::Error &e) {
            jrc = e.code;
            jerr = e.what();
        } catch (const std::exception &e) {
            jrc = FL_EHIP;
            jerr = e.what();
        }
        size_t now_held = worker_held(ctx, d);
        bool over = false;
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            // the job grew its worker's memory past what it was charged
            if (now_held > std::max(held_before, j->bytes)) sv->st.over_estimate++;
            sv->held[me] = now_held;
            sv->busy[me] = 0;
            sv->charge[me] = now_held;
            // past the budget, this worker gives its memory back before the
            // next job
            over = total_charge(sv) > sv->budget;
        }
        if (over && sv->fake_ns <= 0.0) {
            if (!worker_trim(sv, ctx, s, d) && init_err.empty()) init_err = "worker could not recreate its context";
            now_held = worker_held(ctx, d);
        }
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            if (over) sv->st.trims++;
            sv->held[me] = sv->charge[me] = now_held;
            sv->in_use = total_charge(sv);
            size_t all = 0;
            for (size_t h : sv->held) all += h;
            sv->peak_held = std::max(sv->peak_held, all);
            j->t_done = sv->now();
            j->state = jrc == FL_OK ? FL_JOB_DONE : FL_JOB_FAILED;
            j->err = jerr;
            if (jrc == FL_OK) {
                sv->st.completed++;
                sv->st.node_updates += (int64_t)j->n * j->iters;
            } else {
                sv->st.failed++;
            }
            // free the inputs of a finished job; results stay until fetched
            std::vector<int32_t>().swap(j->src);
            std::vector<int32_t>().swap(j->dst);
        }
        sv->cv_done.notify_all();
        sv->cv_work.notify_all();
    }
    d.release();
    if (ctx) fl_destroy(ctx);
    if (s) (void)hipStreamDestroy(s);
}

fl_status server_create(fl_server **out, int device, size_t budget, int32_t slots, double fake_ns)
{
    if (!out || slots < 1 || slots > 64 || budget == 0) return FL_EINVAL;
    *out = nullptr;
    if (fake_ns <= 0.0) {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FL_EINVAL;
    }
    fl_server *sv = new (std::nothrow) fl_server();
    if (!sv) return FL_ENOMEM;
    sv->device = device;
    sv->budget = budget;
    fl_default_tuning(&sv->tuning);
    sv->slots = slots;
    sv->fake_ns = fake_ns;
    sv->held.assign(slots, 0);
    sv->charge.assign(slots, 0);
    sv->busy.assign(slots, 0);
    for (int i = 0; i < slots; ++i) sv->workers.emplace_back(worker, sv, i);
    *out = sv;
    return FL_OK;
}

}  // namespace

extern "C" {

fl_status fl_server_create(fl_server **out, int device, size_t mem_budget_bytes, int32_t max_slots)
{
    return server_create(out, device, mem_budget_bytes, max_slots, 0.0);
}

fl_status fl_server_create_fake(fl_server **out, size_t mem_budget_bytes, int32_t max_slots,
                                double ns_per_node_update)
{
    if (!(ns_per_node_update > 0.0)) return FL_EINVAL;
    return server_create(out, 0, mem_budget_bytes, max_slots, ns_per_node_update);
}

const char *fl_server_last_error(const fl_server *sv) { return sv ? sv->err.c_str() : "null server"; }

fl_status fl_server_submit(fl_server *sv, const fl_job *job, uint64_t *job_id)
{
    if (!sv || !job || !job_id) return FL_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (job->n < 1 || job->m < 0 || job->iters < 0 || !job->x0 || !job->y0 || (job->m > 0 && (!job->src || !job->dst))) {
        sv->err = "fl_server_submit: bad job";
        return FL_EINVAL;
    }
    auto j = std::make_shared<Job>();
    try {
        j->id = sv->next_id++;
        j->n = job->n;
        j->m = job->m;
        j->src.assign(job->src, job->src + job->m);
        j->dst.assign(job->dst, job->dst + job->m);
        j->x.assign(job->x0, job->x0 + job->n);
        j->y.assign(job->y0, job->y0 + job->n);
    } catch (const std::bad_alloc &) {
        sv->err = "fl_server_submit: out of host memory";
        return FL_ENOMEM;
    }
    j->iters = job->iters;
    j->prm = job->params;
    j->t_arrive = sv->now();
    j->bytes = job_bytes(job->n, job->m);
    if (j->bytes > sv->budget) {
        sv->err = "fl_server_submit: job larger than the memory budget";
        return FL_ENOMEM;
    }
    sv->jobs[j->id] = j;
    sv->queue.push_back(j);
    sv->st.submitted++;
    *job_id = j->id;
    sv->cv_work.notify_all();
    return FL_OK;
}

fl_status fl_server_poll(fl_server *sv, uint64_t id, int32_t *state)
{
    if (!sv || !state) return FL_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->jobs.find(id);
    if (it == sv->jobs.end()) return FL_EINVAL;
    *state = it->second->state;
    return FL_OK;
}

fl_status fl_server_wait(fl_server *sv, uint64_t id, double timeout_s, int32_t *state)
{
    if (!sv) return FL_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->jobs.find(id);
    if (it == sv->jobs.end()) return FL_EINVAL;
    auto j = it->second;
    auto done = [&] { return j->state >= FL_JOB_DONE; };
    if (timeout_s < 0) sv->cv_done.wait(lk, done);
    else if (!sv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done)) {
        if (state) *state = j->state;
        return FL_EBUSY;
    }
    if (state) *state = j->state;
    return FL_OK;
}

fl_status fl_server_result(fl_server *sv, uint64_t id, float *x_host, float *y_host, double *times3)
{
    if (!sv) return FL_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->jobs.find(id);
    if (it == sv->jobs.end()) return FL_EINVAL;
    auto j = it->second;
    if (j->state == FL_JOB_QUEUED || j->state == FL_JOB_RUNNING) return FL_EBUSY;
    if (times3) {
        times3[0] = j->t_arrive;
        times3[1] = j->t_start;
        times3[2] = j->t_done;
    }
    if (j->state == FL_JOB_CANCELED) return FL_ECANCELED;
    if (j->state == FL_JOB_FAILED) {
        sv->err = j->err;
        return FL_EHIP;
    }
    if (x_host) std::memcpy(x_host, j->x.data(), 4 * (size_t)j->n);
    if (y_host) std::memcpy(y_host, j->y.data(), 4 * (size_t)j->n);
    return FL_OK;
}

fl_status fl_server_release(fl_server *sv, uint64_t id)
{
    if (!sv) return FL_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->jobs.find(id);
    if (it == sv->jobs.end()) return FL_EINVAL;
    if (it->second->state == FL_JOB_QUEUED || it->second->state == FL_JOB_RUNNING) return FL_EBUSY;
    sv->jobs.erase(it);
    return FL_OK;
}

fl_status fl_server_set_tuning(fl_server *sv, const fl_tuning *tuning)
{
    if (!sv) return FL_EINVAL;
    fl_tuning t;
    if (tuning) t = *tuning;
    else fl_default_tuning(&t);
    try {
        fl::check_tuning(t);
    } catch (const fl::Error &e) {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->err = e.what();
        return e.code;
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->tuning = t;
    return FL_OK;
}

fl_status fl_server_cancel(fl_server *sv, uint64_t id)
{
    if (!sv) return FL_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->jobs.find(id);
    if (it == sv->jobs.end()) return FL_EINVAL;
    auto j = it->second;
    if (j->state != FL_JOB_QUEUED) return FL_EBUSY;  // running jobs finish
    sv->queue.erase(std::remove(sv->queue.begin(), sv->queue.end(), j), sv->queue.end());
    j->state = FL_JOB_CANCELED;
    j->t_done = sv->now();
    sv->st.canceled++;
    sv->cv_done.notify_all();
    sv->cv_work.notify_all();
    return FL_OK;
}

fl_status fl_server_stats_get(fl_server *sv, fl_server_stats *out)
{
    if (!sv || !out) return FL_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    *out = sv->st;
    out->queued = (int64_t)sv->queue.size();
    out->running = (int64_t)(sv->st.admitted - sv->st.completed - sv->st.failed);
    out->bytes_in_use = (int64_t)sv->in_use;
    out->peak_bytes = (int64_t)sv->peak;
    size_t all = 0;
    for (size_t h : sv->held) all += h;
    out->held_bytes = (int64_t)all;
    out->peak_held_bytes = (int64_t)sv->peak_held;
    return FL_OK;
}

void fl_server_destroy(fl_server *sv)
{
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        // queued jobs are cancelled; running ones finish first
        for (auto &j : sv->queue) j->state = FL_JOB_CANCELED;
        sv->queue.clear();
    }
    sv->cv_work.notify_all();
    for (auto &t : sv->workers) t.join();
    delete sv;
}

}  // extern "C"
