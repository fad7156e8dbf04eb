// lp_server.cpp -- request loop for least-model and stable-model queries.
//
// Programs are registered once (host build of the matrix); requests name a
// program and are queued. n_slots worker threads, each with a HIP stream of
// its own, take work from the queue as soon as they are free:
//   * admission: a request is started only when the device bytes it needs
//     (its matrix if not resident, plus its solve buffers) fit in the
//     budget; resident matrices that no running request uses are evicted,
//     least recently used first, to make room; otherwise it waits while later
//     requests that do fit go ahead;
//   * residency: matrices stay on the device between requests (LRU cache);
//   * continuous batching: a free slot takes every waiting least-model
//     request of a small matrix (at most batch_rows rows, within the batch
//     kernel's LDS; up to batch_max requests) and solves them in one launch,
//     one workgroup per program; likewise every waiting stable-model request
//     of a small interpretation matrix (at most 12 negated atoms left after
//     pruning and kStableBatchWords row-words), solved together by
//     lp_stable_models_batch (one launch per product for all of them).
//     Larger requests and a small request with no company run alone on the
//     whole device. Work of different slots overlaps on the device.
// Results are kept until lp_server_take_result.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lp_internal.h"

namespace lp {
namespace {

struct Program {
    int32_t id = 0;
    lp_matrix *m = nullptr;  // host CSR always; device copy while resident
    lp_info info{};
    bool resident = false;
    bool uploading = false;
    int refs = 0;            // admitted requests using the device copy
    int64_t bytes = 0;       // device bytes accounted while resident
    uint64_t last_use = 0;
};

struct Request {
    lp_request_info info{};
    std::vector<uint8_t> model;
    std::vector<uint64_t> accepted;
    int64_t reserved = 0;    // solve buffers accounted while running
};

int64_t words_of(int64_t n) { return (n + 63) / 64; }

// Upper bound of the device bytes of a matrix's layout (every array, with
// the allocator's rounding), before it has been uploaded once.
int64_t matrix_bytes_bound(const lp_info &I) {
    const int64_t W = words_of(I.n_rows);
    double b = 4.0 * (double)I.nnz + 10.0 * (double)I.n_rows + 64.0 * (double)W + 65536.0;
    // stable solves by dirty rows: the transposed matrix (row pointers,
    // entries, start counts, fact rows) is uploaded with the matrix
    if (I.n_neg > 0) b += 4.0 * (double)I.nnz + 12.0 * (double)I.n_rows + 4.0;
    return (int64_t)(1.15 * b) + (1 << 20);
}

// Device bytes of one solve's buffers.
int64_t solve_bytes(const lp_info &I) {
    const int64_t W = words_of(I.n_rows);
    double b;
    if (I.n_neg == 0) {
        b = 16.0 * (double)W + 8.0 * 2048 + 8.0 * (double)I.n_long_rows;
    } else {
        const int64_t Wg = words_of((int64_t)1 << I.n_neg);
        // two interpretation matrices, the accepted mask, the row sets of
        // the dirty-row products (seven bitmaps), the models
        b = 16.0 * (double)I.n_rows * (double)Wg + 8.0 * (double)Wg + (double)I.n_rows + (double)I.n_atoms +
            8.0 * 2048;
    }
    return (int64_t)(1.15 * b) + (1 << 20);
}

}  // namespace
}  // namespace lp

struct lp_server {
    lp_server_config cfg{};
    int device = 0;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work;  // workers: new request or freed memory
    std::condition_variable cv_done;  // waiters: a request completed
    bool stop = false;
    std::vector<std::unique_ptr<lp::Program>> programs;
    std::deque<lp::Request *> pending;
    std::unordered_map<int64_t, std::unique_ptr<lp::Request>> requests;
    std::deque<int64_t> done;
    int64_t next_id = 0;
    int64_t used = 0;                 // accounted device bytes
    int64_t peak_used = 0;
    uint64_t clock = 0;               // LRU ticks
    int64_t n_batches = 0, n_batched = 0, n_alone = 0, n_uploads = 0, n_evictions = 0, n_completed = 0;
    std::atomic<int64_t> n_tunes{0};
    int64_t max_batch_rows = 0;
    std::vector<hipStream_t> streams;
    std::vector<std::thread> workers;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace lp {
namespace {

// Makes room for `need` bytes by evicting idle resident matrices, least
// recently used first. Called with the lock held. Returns false if the
// budget cannot hold `need` even after evicting every idle matrix.
bool make_room(lp_server *s, int64_t need) {
    if (s->used + need <= s->cfg.hbm_budget) return true;
    int64_t idle = 0;
    for (auto &p : s->programs)
        if (p->resident && p->refs == 0 && !p->uploading) idle += p->bytes;
    if (s->used - idle + need > s->cfg.hbm_budget) return false;
    std::vector<Program *> cand;
    for (auto &p : s->programs)
        if (p->resident && p->refs == 0 && !p->uploading) cand.push_back(p.get());
    std::sort(cand.begin(), cand.end(), [](Program *a, Program *b) { return a->last_use < b->last_use; });
    for (Program *p : cand) {
        if (s->used + need <= s->cfg.hbm_budget) break;
        lp_matrix_evict(p->m);
        p->resident = false;
        s->used -= p->bytes;
        p->bytes = 0;
        s->n_evictions++;
    }
    return s->used + need <= s->cfg.hbm_budget;
}

// Admits r if its bytes fit; the lock is held. On success the program is
// referenced and, if it is not resident, marked for upload by the caller.
bool admit(lp_server *s, Request *r, std::vector<Program *> &to_upload) {
    Program *p = s->programs[r->info.program_id].get();
    const bool mine = std::find(to_upload.begin(), to_upload.end(), p) != to_upload.end();
    if (p->uploading && !mine) return false;  // another slot is uploading it
    const int64_t mat = (p->resident || mine) ? 0 : matrix_bytes_bound(p->info);
    const int64_t need = mat + solve_bytes(p->info);
    if (!make_room(s, need)) return false;
    s->used += need;
    s->peak_used = std::max(s->peak_used, s->used);
    r->reserved = need - mat;
    if (!p->resident && !mine) {
        p->uploading = true;
        p->bytes = mat;
        to_upload.push_back(p);
        r->info.built = 1;
    }
    p->refs++;
    p->last_use = ++s->clock;
    return true;
}

// Interpretation matrices of at most this many row-words join stable-model
// batches: full-sweep products of that size cost about a launch; larger ones
// run alone, where products evaluate only the rows that can change.
constexpr int64_t kStableBatchWords = (int64_t)1 << 18;

// Batch kind of a program's requests: 1 least-model batches, 2 stable-model
// batches, 0 alone.
int batch_kind(const lp_server *s, const Program *p) {
    if (s->cfg.batch_max <= 1) return 0;
    if (p->info.n_neg == 0)
        return (p->info.n_rows <= s->max_batch_rows && p->info.n_rows <= s->cfg.batch_rows) ? 1 : 0;
    const int k_eff = p->info.n_neg - p->info.n_pruned;
    if (k_eff > 12) return 0;
    return (int64_t)p->info.n_rows * words_of((int64_t)1 << k_eff) <= kStableBatchWords ? 2 : 0;
}

// Takes the next work item from the queue (lock held): the oldest admissible
// request, and with it every further admissible request of the same batch
// kind (batch_kind), up to batch_max.
bool pick(lp_server *s, std::vector<Request *> &group, std::vector<Program *> &to_upload) {
    group.clear();
    to_upload.clear();
    int kind = 0;
    for (auto it = s->pending.begin(); it != s->pending.end();) {
        Request *r = *it;
        Program *p = s->programs[r->info.program_id].get();
        if (!group.empty() && (kind == 0 || batch_kind(s, p) != kind)) {
            ++it;
            continue;
        }
        if (!admit(s, r, to_upload)) {
            ++it;
            continue;
        }
        if (group.empty()) kind = batch_kind(s, p);
        group.push_back(r);
        it = s->pending.erase(it);
        if (kind == 0 || (int)group.size() >= s->cfg.batch_max) break;
    }
    return !group.empty();
}

void run_group(lp_server *s, hipStream_t st, std::vector<Request *> &group, std::vector<Program *> &to_upload) {
    for (Request *r : group) r->info.t_start = s->now();
    // uploads (outside the lock; the programs are marked, so no other slot touches them)
    std::map<Program *, lp_status> up_rc;
    for (Program *p : to_upload) {
        lp_status rc = lp_matrix_upload(p->m, st);
        up_rc[p] = rc;
        lp_info I{};
        if (!rc) lp_matrix_info(p->m, &I);
        std::lock_guard<std::mutex> lock(s->mu);
        p->uploading = false;
        if (!rc) {
            s->used += I.device_bytes - p->bytes;  // the bound becomes the actual size
            p->bytes = I.device_bytes;
            p->resident = true;
            s->n_uploads++;
        } else {
            s->used -= p->bytes;
            p->bytes = 0;
        }
    }
    auto failed = [&](Program *p) {
        auto it = up_rc.find(p);
        return it != up_rc.end() ? it->second : LP_OK;
    };
    const bool batch = group.size() > 1;
    try {
    if (batch) {
        // one launch for the distinct programs of the group
        std::vector<Program *> progs;
        std::map<Program *, size_t> slot;
        for (Request *r : group) {
            Program *p = s->programs[r->info.program_id].get();
            if (failed(p)) {
                r->info.status = failed(p);
                continue;
            }
            if (!slot.count(p)) {
                slot[p] = progs.size();
                progs.push_back(p);
            }
        }
        std::vector<const lp_matrix *> ms;
        std::vector<std::vector<uint8_t>> models(progs.size());
        std::vector<uint8_t *> mp;
        for (Program *p : progs) {
            ms.push_back(p->m);
            models[mp.size()].assign(std::max(1, p->info.n_atoms), 0);
            mp.push_back(models[mp.size()].data());
        }
        std::vector<int32_t> prods(std::max<size_t>(1, progs.size()), 0);
        // stable-model batches: the accepted masks and model counts too
        const bool stable = !progs.empty() && progs[0]->info.n_neg > 0;
        std::vector<std::vector<uint64_t>> acc(progs.size());
        std::vector<uint64_t *> ap;
        std::vector<int64_t> nm(std::max<size_t>(1, progs.size()), 1);
        if (stable)
            for (Program *p : progs) {
                acc[ap.size()].assign(words_of((int64_t)1 << p->info.n_neg), 0);
                ap.push_back(acc[ap.size()].data());
            }
        lp_status rc = LP_OK;
        if (!progs.empty())
            rc = stable ? lp_stable_models_batch(ms.data(), (int32_t)ms.size(), ap.data(), nm.data(), mp.data(),
                                                 prods.data(), st)
                        : lp_least_model_batch(ms.data(), (int32_t)ms.size(), mp.data(), prods.data(), nullptr, st);
        for (Request *r : group) {
            Program *p = s->programs[r->info.program_id].get();
            if (failed(p)) continue;
            r->info.status = rc;
            r->info.batch_size = (int32_t)group.size();
            if (!rc) {
                const size_t k = slot[p];
                r->model.assign(models[k].begin(), models[k].begin() + p->info.n_atoms);
                r->info.products = prods[k];
                r->info.n_models = nm[k];
                if (stable) r->accepted = acc[k];
            }
        }
    } else {
        Request *r = group[0];
        Program *p = s->programs[r->info.program_id].get();
        r->info.batch_size = 1;
        if (failed(p)) {
            r->info.status = failed(p);
        } else if (p->info.n_neg == 0) {
            r->model.assign(std::max(1, p->info.n_atoms), 0);
            int32_t pr = 0;
            if (s->cfg.tune) {
                // a matrix whose size bucket holds no tuned schedule: tune one (the
                // solve below and later matrices of the bucket use it; slots that
                // meet the same new bucket at once may each tune it)
                lp_schedule cs{};
                int32_t found = 0;
                if (lp_schedule_cache_lookup(p->m, &cs, &found) == LP_OK && found == 0) {
                    lp_schedule best{};
                    if (lp_tune_schedule(p->m, 2, &best, nullptr, nullptr, st) == LP_OK) s->n_tunes++;
                }
            }
            r->info.status = lp_least_model(p->m, r->model.data(), &pr, nullptr, st);
            r->model.resize(p->info.n_atoms);
            r->info.products = pr;
            r->info.n_models = 1;
        } else {
            const int64_t W = words_of((int64_t)1 << p->info.n_neg);
            r->accepted.assign(W, 0);
            r->model.assign(std::max(1, p->info.n_atoms), 0);
            int64_t nm = 0;
            int32_t pr = 0;
            lp_status rc = lp_stable_models(p->m, r->accepted.data(), &nm, r->model.data(), 1, nullptr, &pr, st);
            if (rc == LP_E_TRUNCATED) rc = LP_OK;  // only the first model is kept; the rest is complete
            r->info.status = rc;
            r->model.resize(p->info.n_atoms);
            r->info.products = pr;
            r->info.n_models = nm;
        }
    }
    } catch (const std::bad_alloc &) {
        for (Request *r : group) r->info.status = LP_E_NOMEM;
    }
    // structures a solve attaches to its matrix (wave splits, the stable-solve
    // plan, which takes the place of the buffers the request reserved) become
    // resident bytes as the request's reservation is released
    std::vector<std::pair<Program *, int64_t>> sizes;
    for (Request *r : group) {
        Program *p = s->programs[r->info.program_id].get();
        lp_info I{};
        if (!failed(p) && lp_matrix_info(p->m, &I) == LP_OK) sizes.emplace_back(p, I.device_bytes);
    }
    std::lock_guard<std::mutex> lock(s->mu);
    const double t = s->now();
    for (Request *r : group) {
        Program *p = s->programs[r->info.program_id].get();
        p->refs--;
        s->used -= r->reserved;
        r->reserved = 0;
        r->info.t_done = t;
        s->done.push_back(r->info.request_id);
        s->n_completed++;
    }
    for (auto &ps : sizes) {
        if (!ps.first->resident) continue;
        s->used += ps.second - ps.first->bytes;
        ps.first->bytes = ps.second;
    }
    s->peak_used = std::max(s->peak_used, s->used);
    if (batch) {
        s->n_batches++;
        s->n_batched += (int64_t)group.size();
    } else {
        s->n_alone++;
    }
    s->cv_done.notify_all();
    s->cv_work.notify_all();
}

void worker(lp_server *s, int slot) {
    (void)hipSetDevice(s->device);
    hipStream_t st = s->streams[slot];
    std::vector<Request *> group;
    std::vector<Program *> to_upload;
    for (;;) {
        {
            std::unique_lock<std::mutex> lock(s->mu);
            s->cv_work.wait(lock, [&] { return s->stop || pick(s, group, to_upload); });
            if (s->stop && group.empty()) return;
        }
        run_group(s, st, group, to_upload);
    }
}

}  // namespace
}  // namespace lp

using namespace lp;

extern "C" {

lp_status lp_server_create(const lp_server_config *cfg, lp_server **out) {
    try {
        if (!out) {
            set_error("out must be non-NULL");
            return LP_E_INVAL;
        }
        *out = nullptr;
        std::unique_ptr<lp_server> s(new lp_server());
        if (cfg) s->cfg = *cfg;
        if (s->cfg.n_slots <= 0) s->cfg.n_slots = 4;  // measured: 4 beat 8 at 300 and 1,000 req/s (4 hardware queues per process)
        if (s->cfg.n_slots > 64) {
            set_error("n_slots must be at most 64");
            return LP_E_INVAL;
        }
        if (s->cfg.batch_max <= 0) s->cfg.batch_max = 64;
        if (s->cfg.batch_rows <= 0) s->cfg.batch_rows = 65536;
        int dev = s->cfg.device;
        if (dev < 0 && hipGetDevice(&dev) != hipSuccess) {
            set_error("no HIP device");
            return LP_E_DEVICE;
        }
        s->device = dev;
        if (hipSetDevice(dev) != hipSuccess) {
            set_error("hipSetDevice failed");
            return LP_E_DEVICE;
        }
        if (s->cfg.hbm_budget <= 0) {
            size_t fr = 0, tot = 0;
            if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
                set_error("hipMemGetInfo failed");
                return LP_E_DEVICE;
            }
            s->cfg.hbm_budget = (int64_t)(0.9 * (double)fr);
        }
        s->max_batch_rows = batch_max_rows(dev);
        s->t0 = std::chrono::steady_clock::now();
        for (int i = 0; i < s->cfg.n_slots; ++i) {
            hipStream_t st;
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
                for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
                set_error("hipStreamCreate failed");
                return LP_E_DEVICE;
            }
            s->streams.push_back(st);
        }
        lp_server *raw = s.get();
        for (int i = 0; i < s->cfg.n_slots; ++i) s->workers.emplace_back(worker, raw, i);
        *out = s.release();
        return LP_OK;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return LP_E_NOMEM;
    } catch (...) {
        set_error("unexpected exception");
        return LP_E_INTERNAL;
    }
}

lp_status lp_server_add_program(lp_server *s, int32_t n_atoms, int32_t n_rules, const int32_t *head,
                                const int64_t *body_ptr, const int32_t *body_lit, int32_t *program_id) {
    try {
        if (!s || !program_id) {
            set_error("NULL argument");
            return LP_E_INVAL;
        }
        lp_matrix *m = nullptr;
        lp_status rc = lp_build_matrix(n_atoms, n_rules, head, body_ptr, body_lit, LP_BUILD_HOST_ONLY, nullptr, &m);
        if (rc) return rc;
        std::unique_ptr<Program> p(new Program());
        p->m = m;
        lp_matrix_info(m, &p->info);
        if (p->info.n_neg > LP_MAX_NEG_ATOMS) {
            lp_free_matrix(m);
            set_error("too many negated atoms: " + std::to_string(p->info.n_neg));
            return LP_E_TOO_MANY_GUESSES;
        }
        std::lock_guard<std::mutex> lock(s->mu);
        const int64_t need = matrix_bytes_bound(p->info) + solve_bytes(p->info);
        if (need > s->cfg.hbm_budget) {
            lp_free_matrix(m);
            set_error("program needs " + std::to_string((long long)need) + " device bytes, over the budget");
            return LP_E_NOMEM;
        }
        p->id = (int32_t)s->programs.size();
        *program_id = p->id;
        s->programs.push_back(std::move(p));
        return LP_OK;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return LP_E_NOMEM;
    } catch (...) {
        set_error("unexpected exception");
        return LP_E_INTERNAL;
    }
}

lp_status lp_server_submit(lp_server *s, int32_t program_id, int64_t *request_id) {
    try {
        if (!s) {
            set_error("NULL server");
            return LP_E_INVAL;
        }
        std::lock_guard<std::mutex> lock(s->mu);
        if (program_id < 0 || program_id >= (int32_t)s->programs.size()) {
            set_error("unknown program id");
            return LP_E_INVAL;
        }
        std::unique_ptr<Request> r(new Request());
        const Program &p = *s->programs[program_id];
        r->info.request_id = s->next_id++;
        r->info.program_id = program_id;
        r->info.kind = p.info.n_neg > 0 ? 1 : 0;
        r->info.nnz = p.info.nnz;
        r->info.t_submit = s->now();
        if (request_id) *request_id = r->info.request_id;
        s->pending.push_back(r.get());
        s->requests[r->info.request_id] = std::move(r);
        s->cv_work.notify_one();
        return LP_OK;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return LP_E_NOMEM;
    }
}

lp_status lp_server_wait_any(lp_server *s, int32_t timeout_ms, lp_request_info *out) {
    if (!s || !out) {
        set_error("NULL argument");
        return LP_E_INVAL;
    }
    std::unique_lock<std::mutex> lock(s->mu);
    if (!s->cv_done.wait_for(lock, std::chrono::milliseconds(std::max(0, timeout_ms)),
                             [&] { return !s->done.empty(); })) {
        set_error("no request completed within the timeout");
        return LP_E_TIMEOUT;
    }
    const int64_t id = s->done.front();
    s->done.pop_front();
    *out = s->requests[id]->info;
    return LP_OK;
}

lp_status lp_server_take_result(lp_server *s, int64_t request_id, uint8_t *model, uint64_t *accepted) {
    if (!s) {
        set_error("NULL server");
        return LP_E_INVAL;
    }
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->requests.find(request_id);
    if (it == s->requests.end() || it->second->info.t_done == 0.0) {
        set_error("unknown or unfinished request");
        return LP_E_INVAL;
    }
    Request &r = *it->second;
    if (model && !r.model.empty()) std::memcpy(model, r.model.data(), r.model.size());
    if (accepted && !r.accepted.empty()) std::memcpy(accepted, r.accepted.data(), 8 * r.accepted.size());
    s->requests.erase(it);
    return LP_OK;
}

lp_status lp_server_get_stats(lp_server *s, lp_server_stats *out) {
    if (!s || !out) {
        set_error("NULL argument");
        return LP_E_INVAL;
    }
    std::lock_guard<std::mutex> lock(s->mu);
    lp_server_stats St{};
    St.n_programs = (int32_t)s->programs.size();
    for (auto &p : s->programs) St.n_resident += p->resident ? 1 : 0;
    St.pending = (int64_t)s->pending.size();
    St.completed = s->n_completed;
    St.batches = s->n_batches;
    St.batched_requests = s->n_batched;
    St.alone_requests = s->n_alone;
    St.uploads = s->n_uploads;
    St.evictions = s->n_evictions;
    St.used_bytes = s->used;
    St.peak_used_bytes = s->peak_used;
    St.hbm_budget = s->cfg.hbm_budget;
    St.tunes = s->n_tunes.load();
    *out = St;
    return LP_OK;
}

lp_status lp_server_free(lp_server *s) {
    if (!s) return LP_OK;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    for (auto &t : s->workers) t.join();
    (void)hipSetDevice(s->device);
    for (hipStream_t st : s->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    for (auto &p : s->programs) lp_free_matrix(p->m);
    delete s;
    return LP_OK;
}

}  // extern "C"
