// Ensembles and served requests: many independent problems advanced
// concurrently from one device arena.
//
// Every member is an ordinary jfmg_problem whose workspace is a first-fit range
// of the caller's arena.  A fixed pool of host worker threads advances the
// members one implicit step at a time; each step runs on the member's private
// stream, so the small, latency bound kernels of different members overlap on
// the GPU while one member's host waits for its Arnoldi scalars.  Members share no device memory and every
// kernel reduces in a fixed order, so a member's result does not depend on what
// else runs beside it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "jfmg.h"

namespace {

constexpr size_t ARENA_ALIGN = 256;

struct Member {
    bool used = false;
    bool busy = false;       // a worker is inside jfmg_implicit_step for it
    bool finished = false;   // all steps done, or failed
    jfmg_problem* p = nullptr;
    double* U = nullptr;
    size_t off = 0, len = 0;
    int n_steps = 0, done = 0, target = 0;
    jfmg_status status = JFMG_OK;
    jfmg_stats acc{};
};

}  // namespace

struct jfmg_batch {
    char* arena = nullptr;
    size_t bytes = 0;
    hipStream_t st = nullptr;
    int device = 0;
    std::vector<Member> m;
    std::map<size_t, size_t> free_ranges;   // offset -> length, disjoint, coalesced
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::vector<std::thread> workers;
    std::deque<int> completed;   // finished slots not yet returned by wait_any
    bool background = false, quit = false;
    int rr = 0;                  // round-robin start of the member scan
    std::string err;
};

namespace {

jfmg_status bfail(jfmg_batch* b, jfmg_status s, const std::string& msg)
{
    if (b) b->err = msg;
    return s;
}

// first fit; returns false if no free range holds len bytes
bool arena_take(jfmg_batch* b, size_t len, size_t* off)
{
    len = (len + ARENA_ALIGN - 1) / ARENA_ALIGN * ARENA_ALIGN;
    for (auto it = b->free_ranges.begin(); it != b->free_ranges.end(); ++it) {
        if (it->second < len) continue;
        *off = it->first;
        const size_t rest = it->second - len, at = it->first + len;
        b->free_ranges.erase(it);
        if (rest) b->free_ranges[at] = rest;
        return true;
    }
    return false;
}

void arena_give(jfmg_batch* b, size_t off, size_t len)
{
    len = (len + ARENA_ALIGN - 1) / ARENA_ALIGN * ARENA_ALIGN;
    auto it = b->free_ranges.emplace(off, len).first;
    auto nx = std::next(it);
    if (nx != b->free_ranges.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        b->free_ranges.erase(nx);
    }
    if (it != b->free_ranges.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            b->free_ranges.erase(it);
        }
    }
}

bool runnable(const Member& x) { return x.used && !x.busy && !x.finished && x.done < x.target; }

void accumulate(jfmg_stats& a, const jfmg_stats& s)
{
    a.newton_its += s.newton_its;
    a.gmres_its += s.gmres_its;
    a.lh_evals += s.lh_evals;
    a.jvps += s.jvps;
    for (int l = 0; l < 8; ++l) a.fv_matvecs[l] += s.fv_matvecs[l];
    a.host_syncs += s.host_syncs;
    a.stall_stops += s.stall_stops;
    a.reorth_its += s.reorth_its;
    a.g0_norm = s.g0_norm;
    a.g_norm = s.g_norm;
    a.seconds += s.seconds;
    a.reached_rtol = a.reached_rtol > s.reached_rtol ? a.reached_rtol : s.reached_rtol;
    if (a.status == JFMG_OK) a.status = s.status;
}

void worker_main(jfmg_batch* b)
{
    (void)hipSetDevice(b->device);
    std::unique_lock<std::mutex> lk(b->mu);
    for (;;) {
        int pick = -1;
        b->cv_work.wait(lk, [&] {
            if (b->quit) return true;
            const int n = (int)b->m.size();
            for (int i = 0; i < n; ++i) {
                const int s = (b->rr + i) % n;
                if (runnable(b->m[s])) { pick = s; return true; }
            }
            return false;
        });
        if (b->quit) return;
        b->rr = (pick + 1) % (int)b->m.size();
        Member& x = b->m[pick];
        x.busy = true;
        jfmg_problem* p = x.p;
        double* U = x.U;
        lk.unlock();
        jfmg_stats s{};
        const jfmg_status rc = jfmg_implicit_step(p, U, &s);
        lk.lock();
        s.status = rc;
        accumulate(x.acc, s);
        x.busy = false;
        if (rc != JFMG_OK) {
            x.status = rc;
            x.finished = true;
        } else {
            x.done++;
            if (x.done >= x.n_steps) x.finished = true;
        }
        if (x.finished) b->completed.push_back(pick);
        b->cv_done.notify_all();
        b->cv_work.notify_all();
    }
}

bool any_active(const jfmg_batch* b)
{
    for (const Member& x : b->m)
        if (x.busy || runnable(x)) return true;
    return false;
}

}  // namespace

extern "C" {

jfmg_status jfmg_batch_create(size_t arena_bytes, void* arena, int max_members, int workers, void* hip_stream,
                              jfmg_batch** out)
{
    if (!out || !arena || arena_bytes == 0 || max_members <= 0) return JFMG_EINVAL;
    *out = nullptr;
    if (((uintptr_t)arena & (ARENA_ALIGN - 1)) != 0) return JFMG_EINVAL;
    if (workers <= 0) workers = std::min(max_members, 8);
    workers = std::min(workers, 64);
    jfmg_batch* b = new jfmg_batch();
    b->arena = (char*)arena;
    b->bytes = arena_bytes / ARENA_ALIGN * ARENA_ALIGN;
    b->st = (hipStream_t)hip_stream;
    if (hipGetDevice(&b->device) != hipSuccess) { delete b; return JFMG_EDEVICE; }
    b->m.resize(max_members);
    b->free_ranges[0] = b->bytes;
    for (int i = 0; i < workers; ++i) b->workers.emplace_back(worker_main, b);
    *out = b;
    return JFMG_OK;
}

jfmg_status jfmg_batch_destroy(jfmg_batch* b)
{
    if (!b) return JFMG_OK;
    {
        std::unique_lock<std::mutex> lk(b->mu);
        b->background = false;
        for (Member& x : b->m) x.target = x.done;   // no new steps
        b->cv_done.wait(lk, [&] { return !any_active(b); });
        b->quit = true;
        b->cv_work.notify_all();
    }
    for (std::thread& t : b->workers) t.join();
    for (Member& x : b->m)
        if (x.used) (void)jfmg_destroy_problem(x.p);
    delete b;
    return JFMG_OK;
}

jfmg_status jfmg_batch_admit(jfmg_batch* b, const jfmg_config* cfg, const jfmg_perturbation* pert, double* U,
                             int n_steps, int* slot)
{
    if (!b || !cfg || !U || !slot || n_steps < 0) return bfail(b, JFMG_EINVAL, "null argument or negative steps");
    *slot = -1;
    size_t need = 0;
    jfmg_status s = jfmg_workspace_bytes(cfg, &need);
    if (s) return bfail(b, s, std::string("invalid configuration: ") + jfmg_last_error(nullptr));
    int free_slot = -1;
    size_t off = 0;
    {
        std::lock_guard<std::mutex> lk(b->mu);
        for (int i = 0; i < (int)b->m.size(); ++i)
            if (!b->m[i].used) { free_slot = i; break; }
        if (free_slot < 0) return bfail(b, JFMG_ENOMEM, "no free member slot");
        if (!arena_take(b, need, &off)) return bfail(b, JFMG_ENOMEM, "arena has no free range of that size");
        b->m[free_slot].used = true;   // reserved; not runnable until target is set below
        b->m[free_slot].finished = true;
    }
    jfmg_problem* p = nullptr;
    s = jfmg_create_problem(cfg, b->arena + off, need, b->st, &p);
    std::string why = s ? std::string("member creation failed: ") + jfmg_last_error(nullptr) : std::string();
    if (!s && pert) {   // stream ordered before the member's first step (which synchronizes b->st)
        s = jfmg_initial_state(p, pert, U);
        if (s) why = std::string("initial state failed: ") + jfmg_last_error(p);
        if (s) (void)jfmg_destroy_problem(p);
    }
    std::lock_guard<std::mutex> lk(b->mu);
    Member& x = b->m[free_slot];
    if (s) {
        arena_give(b, off, need);
        x = Member();
        return bfail(b, s, why);
    }
    x.p = p;
    x.U = U;
    x.off = off;
    x.len = need;
    x.n_steps = n_steps;
    x.done = 0;
    x.status = JFMG_OK;
    x.acc = jfmg_stats{};
    x.finished = (n_steps == 0);
    x.target = b->background ? n_steps : 0;
    if (x.finished) b->completed.push_back(free_slot);
    *slot = free_slot;
    b->cv_work.notify_all();
    return JFMG_OK;
}

jfmg_problem* jfmg_batch_member(jfmg_batch* b, int slot)
{
    if (!b || slot < 0 || slot >= (int)b->m.size()) return nullptr;
    std::lock_guard<std::mutex> lk(b->mu);
    return b->m[slot].used ? b->m[slot].p : nullptr;
}

jfmg_status jfmg_batch_run(jfmg_batch* b, int max_steps)
{
    if (!b) return JFMG_EINVAL;
    if (b->st && hipStreamSynchronize(b->st) != hipSuccess) return bfail(b, JFMG_EDEVICE, "stream synchronize failed");
    std::unique_lock<std::mutex> lk(b->mu);
    if (b->background) return bfail(b, JFMG_ESTATE, "jfmg_batch_run while background progress is on");
    for (Member& x : b->m)
        if (x.used && !x.finished) x.target = max_steps > 0 ? std::min(x.n_steps, x.done + max_steps) : x.n_steps;
    b->cv_work.notify_all();
    b->cv_done.wait(lk, [&] { return !any_active(b); });
    return JFMG_OK;
}

jfmg_status jfmg_batch_start(jfmg_batch* b)
{
    if (!b) return JFMG_EINVAL;
    if (b->st && hipStreamSynchronize(b->st) != hipSuccess) return bfail(b, JFMG_EDEVICE, "stream synchronize failed");
    std::lock_guard<std::mutex> lk(b->mu);
    b->background = true;
    for (Member& x : b->m)
        if (x.used) x.target = x.n_steps;
    b->cv_work.notify_all();
    return JFMG_OK;
}

jfmg_status jfmg_batch_stop(jfmg_batch* b)
{
    if (!b) return JFMG_EINVAL;
    std::unique_lock<std::mutex> lk(b->mu);
    b->background = false;
    for (Member& x : b->m) x.target = x.done;
    b->cv_done.wait(lk, [&] { return !any_active(b); });
    return JFMG_OK;
}

jfmg_status jfmg_batch_wait_any(jfmg_batch* b, double timeout_s, int* slot)
{
    if (!b || !slot) return JFMG_EINVAL;
    *slot = -1;
    std::unique_lock<std::mutex> lk(b->mu);
    auto ready = [&] { return !b->completed.empty() || !any_active(b); };
    if (timeout_s < 0) b->cv_done.wait(lk, ready);
    else b->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready);
    if (!b->completed.empty()) {
        *slot = b->completed.front();
        b->completed.pop_front();
    }
    return JFMG_OK;
}

jfmg_status jfmg_batch_poll(jfmg_batch* b, int slot, int* finished, int* steps_done, jfmg_stats* stats)
{
    if (!b || slot < 0 || slot >= (int)b->m.size()) return bfail(b, JFMG_EINVAL, "bad slot");
    std::lock_guard<std::mutex> lk(b->mu);
    const Member& x = b->m[slot];
    if (!x.used) return bfail(b, JFMG_EINVAL, "slot is not in use");
    if (finished) *finished = x.finished && !x.busy ? 1 : 0;
    if (steps_done) *steps_done = x.done;
    if (stats) {
        *stats = x.acc;
        stats->status = x.status;
    }
    return x.status;
}

jfmg_status jfmg_batch_retire(jfmg_batch* b, int slot)
{
    if (!b || slot < 0 || slot >= (int)b->m.size()) return bfail(b, JFMG_EINVAL, "bad slot");
    jfmg_problem* p = nullptr;
    {
        std::lock_guard<std::mutex> lk(b->mu);
        Member& x = b->m[slot];
        if (!x.used) return bfail(b, JFMG_EINVAL, "slot is not in use");
        if (x.busy) return bfail(b, JFMG_ESTATE, "member is being advanced");
        p = x.p;
        arena_give(b, x.off, x.len);
        x = Member();
        b->completed.erase(std::remove(b->completed.begin(), b->completed.end(), slot), b->completed.end());
    }
    return jfmg_destroy_problem(p);
}

size_t jfmg_batch_arena_free(jfmg_batch* b)
{
    if (!b) return 0;
    std::lock_guard<std::mutex> lk(b->mu);
    size_t best = 0;
    for (const auto& r : b->free_ranges) best = std::max(best, r.second);
    return best;
}

const char* jfmg_batch_last_error(const jfmg_batch* b) { return b ? b->err.c_str() : "null batch"; }

}  // extern "C"
