// bbe_batch.hip -- batches of uneven Monte-Carlo requests: request
// descriptors and the work list on the device, launch-shape autotuning and
// a captured HIP graph of the whole launch sequence (include/bbe.h).
#include "abi_internal.hpp"

#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <new>
#include <vector>

using namespace bbe_abi;

namespace {

struct Shape {
    int waves_per_block;
    int sims_per_item;  // multiple of 64: one work item = sims_per_item / 64 generations
    int cu_share;       // workgroups per CU: the resident capacity divided by cu_share (1, 2)
};

// Autotune results per (device, size class of the work list), in memory and
// in a JSON file (see tune_cache_path) keyed by the device, the library's
// kernel sources and the size class.
std::mutex g_tune_mu;
std::map<std::pair<int, int>, Shape> g_tuned;
bool g_tune_file_read = false;

struct Group {
    uint32_t first;  // its items: chunks[first .. first + count)
    uint32_t count;
    bool paced;      // the items of races with a time term of R
};

struct Work {
    std::vector<bbe::Chunk> chunks;
    std::vector<Group> groups;
};

// Expected ticks until the request's simulations end (used only to order
// the work list): remaining distance over a typical free step.
double expected_ticks(const bbe::ReqDesc& r) {
    const int n = r.rc.n;
    double lead = 0.0, last = 1e30, fast = 0.0, slow = 1e30;
    for (int k = 0; k < n; ++k) {
        lead = std::max(lead, (double)r.d0[k]);
        last = std::min(last, (double)r.d0[k]);
    }
    for (int c = 0; c < n; ++c) {
        double m = (double)r.rc.elo[c] + 0x1p15 * (double)r.rc.espan16[c];
        fast = std::max(fast, m);
        slow = std::min(slow, m);
    }
    double first = ((double)r.rc.L - lead) / std::max(fast, 1e-30);
    double all = ((double)r.rc.L - last) / std::max(slow, 1e-30);
    double f = n > 1 ? (double)(r.stop_after - 1) / (double)(n - 1) : 0.0;
    return first + f * (all - first);
}

Work build_work(const std::vector<bbe::ReqDesc>& reqs, int sims_per_item) {
    Work w;
    // (paced, expected work) per item: plain items first, each launch's
    // items largest first (competitor-steps: ticks x competitors x sims)
    std::vector<std::pair<std::pair<bool, double>, bbe::Chunk>> items;
    for (size_t r = 0; r < reqs.size(); ++r) {
        const double ticks = expected_ticks(reqs[r]);
        const bool paced = reqs[r].pace.paced != 0;
        for (uint64_t first = 0; first < reqs[r].n_sims; first += (uint64_t)sims_per_item) {
            bbe::Chunk c;
            c.req = (uint32_t)r;
            c.first = (uint32_t)first;
            c.count = (uint32_t)std::min<uint64_t>((uint64_t)sims_per_item,
                                                   reqs[r].n_sims - first);
            c.n = (uint32_t)reqs[r].rc.n;
            items.push_back({{paced, ticks * c.n * c.count}, c});
        }
    }
    std::stable_sort(items.begin(), items.end(), [](const auto& a, const auto& b) {
        if (a.first.first != b.first.first) return !a.first.first;
        return a.first.second > b.first.second;
    });
    w.chunks.reserve(items.size());
    for (auto& it : items) {
        const bool paced = it.first.first;
        if (w.groups.empty() || w.groups.back().paced != paced)
            w.groups.push_back({(uint32_t)w.chunks.size(), 0u, paced});
        w.groups.back().count += 1;
        w.chunks.push_back(it.second);
    }
    return w;
}

// ---------------------------------------------------------------------------
// Persistent tuning cache.  A JSON file of entries {device, kernels,
// size_class, waves_per_block, sims_per_item, cu_share}, one per line:
// $BBE_TUNE_CACHE if set (empty: no file), else
// $XDG_CACHE_HOME/bbe/tune.json or $HOME/.cache/bbe/tune.json.  An entry
// applies to the device it was tuned on (architecture, name, CU count) and
// to the kernel sources it was tuned with (a hash fixed at build time).
// ---------------------------------------------------------------------------
#ifndef BBE_KERNEL_HASH
#define BBE_KERNEL_HASH "unknown"
#endif

std::string tune_cache_path() {
    if (const char* p = std::getenv("BBE_TUNE_CACHE")) return p;
    if (const char* x = std::getenv("XDG_CACHE_HOME"); x && *x)
        return std::string(x) + "/bbe/tune.json";
    if (const char* h = std::getenv("HOME"); h && *h) return std::string(h) + "/.cache/bbe/tune.json";
    return "";
}

std::string device_key(int dev) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    char buf[400];
    std::snprintf(buf, sizeof buf, "%s/%s/%d", prop.gcnArchName, prop.name,
                  prop.multiProcessorCount);
    for (char* c = buf; *c; ++c)
        if (*c == '"' || *c == '\\' || (unsigned char)*c < 32) *c = '_';
    return buf;
}

struct TuneEntry {
    std::string device, kernels;
    int size_class;
    Shape shape;
};

std::vector<TuneEntry> read_tune_file(const std::string& path) {
    std::vector<TuneEntry> out;
    FILE* f = path.empty() ? nullptr : std::fopen(path.c_str(), "r");
    if (!f) return out;
    char line[1024];
    while (std::fgets(line, sizeof line, f)) {
        char dev[400], ker[80];
        TuneEntry e;
        if (std::sscanf(line,
                        " {\"device\": \"%399[^\"]\", \"kernels\": \"%79[^\"]\", \"size_class\": %d, "
                        "\"waves_per_block\": %d, \"sims_per_item\": %d, \"cu_share\": %d}",
                        dev, ker, &e.size_class, &e.shape.waves_per_block,
                        &e.shape.sims_per_item, &e.shape.cu_share) == 6) {
            e.device = dev;
            e.kernels = ker;
            out.push_back(e);
        }
    }
    std::fclose(f);
    return out;
}

bool valid_shape(const Shape& s) {
    return (s.waves_per_block == 1 || s.waves_per_block == 2 || s.waves_per_block == 4) &&
           s.sims_per_item >= 64 && s.sims_per_item <= 65536 && s.sims_per_item % 64 == 0 &&
           (s.cu_share == 1 || s.cu_share == 2);
}

// Loads this device's entries for these kernel sources (once per process).
// Call with g_tune_mu held.
void load_tune_cache(int dev) {
    if (g_tune_file_read) return;
    g_tune_file_read = true;
    const std::string me = device_key(dev);
    for (const TuneEntry& e : read_tune_file(tune_cache_path()))
        if (e.device == me && e.kernels == BBE_KERNEL_HASH && valid_shape(e.shape))
            g_tuned[{dev, e.size_class}] = e.shape;
}

// Adds or replaces one entry in the file (best effort: a file that cannot be
// written leaves the in-memory result in place).  Call with g_tune_mu held.
void store_tune_entry(int dev, int size_class, const Shape& sh) {
    const std::string path = tune_cache_path();
    if (path.empty()) return;
    const std::string me = device_key(dev);
    std::vector<TuneEntry> all = read_tune_file(path);
    bool replaced = false;
    for (TuneEntry& e : all)
        if (e.device == me && e.kernels == BBE_KERNEL_HASH && e.size_class == size_class) {
            e.shape = sh;
            replaced = true;
        }
    if (!replaced) all.push_back({me, BBE_KERNEL_HASH, size_class, sh});
    // create the directory one level up (the usual .../bbe/ folder)
    const size_t slash = path.find_last_of('/');
    if (slash != std::string::npos && slash > 0) (void)mkdir(path.substr(0, slash).c_str(), 0755);
    const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\"entries\": [\n");
    for (size_t i = 0; i < all.size(); ++i)
        std::fprintf(f,
                     "  {\"device\": \"%s\", \"kernels\": \"%s\", \"size_class\": %d, "
                     "\"waves_per_block\": %d, \"sims_per_item\": %d, \"cu_share\": %d}%s\n",
                     all[i].device.c_str(), all[i].kernels.c_str(), all[i].size_class,
                     all[i].shape.waves_per_block, all[i].shape.sims_per_item,
                     all[i].shape.cu_share, i + 1 < all.size() ? "," : "");
    std::fprintf(f, "]}\n");
    const bool good = std::fclose(f) == 0;
    if (good) (void)std::rename(tmp.c_str(), path.c_str());
    else (void)std::remove(tmp.c_str());
}

int size_class(size_t n_chunks) {
    int c = 0;
    while (n_chunks > 1) {
        n_chunks >>= 1;
        ++c;
    }
    return c;
}

}  // namespace

struct bbe_batch_plan {
    int device = 0;
    int n_reqs = 0;
    bbe::ReqDesc* d_reqs = nullptr;
    bbe::Chunk* d_chunks = nullptr;
    size_t chunk_cap = 0;
    uint32_t* d_queue = nullptr;  // one work-queue head per group
    uint32_t n_chunks = 0;
    std::vector<Group> groups;
    std::vector<int> grids;
    uint32_t k0 = 0, k1 = 0;
    unsigned long long* wins = nullptr;
    double* probs = nullptr;
    unsigned long long* steps = nullptr;
    Shape shape{4, 64, 1};
    int item_sims = 64;  // simulations per work item in use (>= shape.sims_per_item)
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<bbe::ReqDesc> host_reqs;
};

namespace {

hipError_t enqueue(bbe_batch_plan* p, hipStream_t s) {
    hipError_t e;
    if ((e = bbe::launch_zero_u64(p->wins, p->n_reqs * bbe::kMaxN, s)) != hipSuccess) return e;
    if (p->steps && (e = bbe::launch_zero_u64(p->steps, 1, s)) != hipSuccess) return e;
    if ((e = bbe::launch_fill_u32(p->d_queue, 0u, (int)p->groups.size(), s)) != hipSuccess)
        return e;
    for (size_t g = 0; g < p->groups.size(); ++g) {
        const Group& gr = p->groups[g];
        bbe::BatchArgs a;
        a.reqs = p->d_reqs;
        a.chunks = p->d_chunks + gr.first;
        a.n_chunks = gr.count;
        a.queue = p->d_queue + g;
        a.wins = p->wins;
        a.steps = p->steps;
        a.k0 = p->k0;
        a.k1 = p->k1;
        if ((e = bbe::launch_batch_mc(a, p->shape.waves_per_block, p->grids[g], gr.paced, s)) !=
            hipSuccess)
            return e;
    }
    if (p->probs &&
        (e = bbe::launch_batch_probs(p->wins, p->d_reqs, p->n_reqs, p->probs, s)) != hipSuccess)
        return e;
    return hipSuccess;
}

// Work items of a batch: ceil(n_sims / 64) generations per request.
uint64_t generation_count(const std::vector<bbe::ReqDesc>& reqs) {
    uint64_t g = 0;
    for (const bbe::ReqDesc& r : reqs) g += (r.n_sims + 63u) / 64u;
    return g;
}

// Simulations per work item actually used for a shape: the shape's own,
// raised (in whole generations) so that a batch has at most kMaxItems
// items: a batch of very large requests gets fewer, longer items instead of
// a work list of tens of millions.
constexpr uint64_t kMaxItems = 1u << 20;
int item_sims(const std::vector<bbe::ReqDesc>& reqs, int sims_per_item) {
    const uint64_t gens = generation_count(reqs);
    const uint64_t min_gens = (gens + kMaxItems - 1) / kMaxItems;
    return (int)std::max<uint64_t>((uint64_t)sims_per_item, 64u * min_gens);
}

int upload_work(bbe_batch_plan* p, const Shape& sh, const std::vector<bbe::ReqDesc>& reqs) {
    const int per_item = item_sims(reqs, sh.sims_per_item);
    Work w = build_work(reqs, per_item);
    if (w.chunks.size() > p->chunk_cap) {
        if (p->d_chunks) (void)hipFree(p->d_chunks);
        p->d_chunks = nullptr;
        p->chunk_cap = 0;
        if (dev_alloc(&p->d_chunks, w.chunks.size() * sizeof(bbe::Chunk)) != hipSuccess)
            return fail(BBE_ENOMEM, "device allocation of the work list failed");
        p->chunk_cap = w.chunks.size();
    }
    hipError_t e = BBE_HIP(hipMemcpy(p->d_chunks, w.chunks.data(),
                                     w.chunks.size() * sizeof(bbe::Chunk), hipMemcpyHostToDevice));
    if (e != hipSuccess) return hip_fail(e, "copying the work list");
    p->n_chunks = (uint32_t)w.chunks.size();
    p->shape = sh;
    p->item_sims = per_item;
    p->groups = w.groups;
    p->grids.clear();
    const int cus = device_cus();
    for (const Group& g : w.groups) {
        // resident capacity (or a share of it), but no more waves than the
        // launch has items
        long cap = std::max(1L, (long)bbe::batch_blocks_per_cu(sh.waves_per_block, g.paced) /
                                    sh.cu_share) *
                   cus;
        long need = ((long)g.count + sh.waves_per_block - 1) / sh.waves_per_block;
        p->grids.push_back((int)std::max(1L, std::min(cap, need)));
    }
    return BBE_OK;
}

void destroy(bbe_batch_plan* p) {
    if (!p) return;
    if (p->d_reqs || p->d_chunks || p->d_queue || p->exec) (void)hipDeviceSynchronize();
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    if (p->d_reqs) (void)hipFree(p->d_reqs);
    if (p->d_chunks) (void)hipFree(p->d_chunks);
    if (p->d_queue) (void)hipFree(p->d_queue);
    delete p;
}

int fill_desc(const bbe_request& q, int idx, bbe::ReqDesc& d) {
    if (!q.race) return fail(BBE_EINVAL, "request %d: race is NULL", idx);
    std::memset(&d, 0, sizeof d);
    d.rc = q.race->rc;
    d.pace = q.race->pace;
    int rc = check_state(q.race, q.state, d.d0, d.s0, d.id0, &d.t0);
    if (rc != BBE_OK) return fail(rc, "request %d: %s", idx, g_err.c_str());
    d.request = q.request;
    d.sim_begin = q.sim_begin;
    d.n_sims = q.n_sims;
    d.stop_after = q.stop_after == 0 ? q.race->n : q.stop_after;
    return BBE_OK;
}

}  // namespace

BBE_API int bbe_batch_plan_create(const bbe_request* reqs, int n_reqs, uint64_t seed,
                                  uint64_t* win_counts, double* probs, uint64_t* step_count,
                                  unsigned flags, void* stream, bbe_batch_plan** out) {
    if (!out) return fail(BBE_EINVAL, "out is NULL");
    *out = nullptr;
    if (!reqs || n_reqs < 1) return fail(BBE_EINVAL, "need n_reqs >= 1 requests");
    if (!win_counts) return fail(BBE_EINVAL, "win_counts is NULL");
    bbe_batch_plan* p = new (std::nothrow) bbe_batch_plan();
    if (!p) return fail(BBE_ENOMEM, "out of host memory");
    p->n_reqs = n_reqs;
    p->host_reqs.resize(n_reqs);
    for (int i = 0; i < n_reqs; ++i) {
        const bbe_request& q = reqs[i];
        int rc = fill_desc(q, i, p->host_reqs[i]);
        if (rc != BBE_OK) {
            destroy(p);
            return rc;
        }
        if (q.n_sims == 0) {
            destroy(p);
            return fail(BBE_EINVAL, "request %d: n_sims must be >= 1", i);
        }
        if ((uint64_t)q.sim_begin + q.n_sims > 0x100000000ull) {
            destroy(p);
            return fail(BBE_EINVAL, "request %d: sim_begin + n_sims exceeds 2^32", i);
        }
        if (q.stop_after < 0 || q.stop_after > q.race->n) {
            destroy(p);
            return fail(BBE_EINVAL, "request %d: stop_after = %d outside 0..%d", i,
                        q.stop_after, q.race->n);
        }
    }
    p->k0 = (uint32_t)seed;
    p->k1 = (uint32_t)(seed >> 32);
    p->wins = reinterpret_cast<unsigned long long*>(win_counts);
    p->probs = probs;
    p->steps = reinterpret_cast<unsigned long long*>(step_count);
    (void)hipGetDevice(&p->device);

    hipError_t e;
    if (dev_alloc(&p->d_reqs, sizeof(bbe::ReqDesc) * n_reqs) != hipSuccess ||
        dev_alloc(&p->d_queue, sizeof(uint32_t) * bbe::kMaxN) != hipSuccess) {
        destroy(p);
        return fail(BBE_ENOMEM, "device allocation of the request table failed");
    }
    if ((e = BBE_HIP(hipMemcpy(p->d_reqs, p->host_reqs.data(), sizeof(bbe::ReqDesc) * n_reqs,
                               hipMemcpyHostToDevice))) != hipSuccess) {
        destroy(p);
        return hip_fail(e, "copying the request table");
    }
    if ((e = BBE_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking))) !=
        hipSuccess) {
        destroy(p);
        return hip_fail(e, "creating the capture stream");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);

    // Launch shape: tuned on this batch, or from the cache, or the default.
    Shape best{4, 64, 1};
    std::pair<int, int> key{p->device, size_class(generation_count(p->host_reqs))};
    bool have = false;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_tune_cache(p->device);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            best = it->second;
            have = true;
        }
    }
    if ((flags & BBE_PLAN_AUTOTUNE) && !have) {
        const Shape cands[] = {{4, 64, 1},  {2, 64, 1},  {1, 64, 1}, {4, 128, 1},
                               {2, 128, 1}, {1, 128, 1}, {4, 256, 1}, {4, 64, 2},
                               {1, 64, 2}};
        // Candidates are timed on the batch itself, or -- for a batch of
        // more than kTuneGens generations -- on the same requests with their
        // simulation counts scaled down to about that much work.
        constexpr uint64_t kTuneGens = 1u << 16;
        std::vector<bbe::ReqDesc> tune = p->host_reqs;
        const uint64_t gens = generation_count(tune);
        if (gens > kTuneGens)
            for (bbe::ReqDesc& r : tune)
                r.n_sims = (uint32_t)std::max<uint64_t>(1u, (uint64_t)r.n_sims * kTuneGens / gens);
        float best_ms = 1e30f;
        hipEvent_t ev0, ev1;
        (void)hipEventCreate(&ev0);
        (void)hipEventCreate(&ev1);
        for (const Shape& c : cands) {
            int rc = upload_work(p, c, tune);
            if (rc != BBE_OK) {
                (void)hipEventDestroy(ev0);
                (void)hipEventDestroy(ev1);
                destroy(p);
                return rc;
            }
            float ms_sum = 0.0f;
            bool okc = true;
            for (int rep = 0; rep < 3 && okc; ++rep) {
                (void)hipEventRecord(ev0, s);
                okc = enqueue(p, s) == hipSuccess;
                (void)hipEventRecord(ev1, s);
                (void)hipEventSynchronize(ev1);
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, ev0, ev1);
                if (rep > 0) ms_sum += ms;  // first run warms up
            }
            if (okc && ms_sum < best_ms) {
                best_ms = ms_sum;
                best = c;
            }
        }
        (void)hipEventDestroy(ev0);
        (void)hipEventDestroy(ev1);
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[key] = best;
        store_tune_entry(p->device, key.second, best);
    }
    int rc = upload_work(p, best, p->host_reqs);
    if (rc != BBE_OK) {
        destroy(p);
        return rc;
    }

    // Capture clear -> queue reset -> persistent kernel -> probabilities.
    if ((e = BBE_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal))) !=
        hipSuccess) {
        destroy(p);
        return hip_fail(e, "beginning graph capture");
    }
    hipError_t ee = enqueue(p, p->cap_stream);
    e = hipStreamEndCapture(p->cap_stream, &p->graph);
    if (ee != hipSuccess || e != hipSuccess) {
        destroy(p);
        return hip_fail(ee != hipSuccess ? ee : e, "capturing the launch sequence");
    }
    if ((e = BBE_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0))) !=
        hipSuccess) {
        destroy(p);
        return hip_fail(e, "instantiating the graph");
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) {
        destroy(p);
        return hip_fail(e, "synchronizing after plan set-up");
    }
    *out = p;
    return ok();
}

BBE_API int bbe_batch_plan_launch(bbe_batch_plan* plan, void* stream) {
    if (!plan || !plan->exec) return fail(BBE_EINVAL, "plan is NULL");
    hipError_t e = BBE_HIP(hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)));
    if (e != hipSuccess) return hip_fail(e, "launching the plan graph");
    return ok();
}

BBE_API int bbe_batch_plan_set_states(bbe_batch_plan* plan, const bbe_state* states,
                                      void* stream) {
    if (!plan || !plan->exec) return fail(BBE_EINVAL, "plan is NULL");
    if (!states) return fail(BBE_EINVAL, "states is NULL");
    const int n_reqs = plan->n_reqs;
    // validate every state before touching the plan
    std::vector<float> d0((size_t)n_reqs * bbe::kMaxN), s0((size_t)n_reqs * bbe::kMaxN);
    std::vector<uint8_t> id0((size_t)n_reqs * bbe::kMaxN);
    std::vector<uint32_t> t0(n_reqs);
    for (int r = 0; r < n_reqs; ++r) {
        const bbe::ReqDesc& q = plan->host_reqs[r];
        int rc = check_state(q.rc.n, q.rc.L, &states[r], &d0[(size_t)r * bbe::kMaxN],
                             &s0[(size_t)r * bbe::kMaxN], &id0[(size_t)r * bbe::kMaxN], &t0[r]);
        if (rc != BBE_OK) return fail(rc, "request %d: %s", r, g_err.c_str());
    }
    for (int r = 0; r < n_reqs; ++r) {
        bbe::ReqDesc& q = plan->host_reqs[r];
        const int n = q.rc.n;
        std::memcpy(q.d0, &d0[(size_t)r * bbe::kMaxN], n * sizeof(float));
        std::memcpy(q.s0, &s0[(size_t)r * bbe::kMaxN], n * sizeof(float));
        std::memcpy(q.id0, &id0[(size_t)r * bbe::kMaxN], n);
        q.t0 = t0[r];
    }
    // ordered after earlier launches on `stream`; the pageable source is
    // consumed before the call returns
    hipError_t e = BBE_HIP(hipMemcpyAsync(plan->d_reqs, plan->host_reqs.data(),
                                          sizeof(bbe::ReqDesc) * n_reqs, hipMemcpyHostToDevice,
                                          static_cast<hipStream_t>(stream)));
    if (e != hipSuccess) return hip_fail(e, "copying the request table");
    return ok();
}

BBE_API int bbe_batch_plan_info(const bbe_batch_plan* plan, int* waves_per_block, int* grid,
                                int* sims_per_item, int* n_items) {
    if (!plan) return fail(BBE_EINVAL, "plan is NULL");
    if (waves_per_block) *waves_per_block = plan->shape.waves_per_block;
    if (grid) {
        int g = 0;
        for (int x : plan->grids) g = std::max(g, x);
        *grid = g;
    }
    if (sims_per_item) *sims_per_item = plan->item_sims;
    if (n_items) *n_items = (int)plan->n_chunks;
    return ok();
}

BBE_API void bbe_batch_plan_free(bbe_batch_plan* plan) { destroy(plan); }

namespace {

// One request of an in-play state batch: the descriptor bbe_prefix_batch and
// bbe_prefix_batch_noalloc hand to the kernel.
int fill_prefix_desc(const bbe_request& q, uint32_t sim, float target, int idx,
                     bbe::ReqDesc& d) {
    int rc = fill_desc(q, idx, d);
    if (rc != BBE_OK) return rc;
    if (!std::isfinite(target) || !(target < q.race->L))
        return fail(BBE_EINVAL, "request %d: target must be finite and < track length", idx);
    d.prefix_sim = sim;
    d.target = target;
    return BBE_OK;
}

}  // namespace

BBE_API int bbe_prefix_batch(const bbe_request* reqs, const uint32_t* sims, const float* targets,
                             int n, uint64_t seed, uint32_t* tick_out, float* pos_out,
                             float* prev_out, void* stream) {
    if (!reqs || !sims || !targets || n < 1) return fail(BBE_EINVAL, "bad batch arguments");
    if (!tick_out || !pos_out || !prev_out) return fail(BBE_EINVAL, "NULL output");
    std::vector<bbe::ReqDesc> h(n);
    for (int i = 0; i < n; ++i) {
        int rc = fill_prefix_desc(reqs[i], sims[i], targets[i], i, h[i]);
        if (rc != BBE_OK) return rc;
    }
    bbe::ReqDesc* d = nullptr;
    if (dev_alloc(&d, sizeof(bbe::ReqDesc) * n) != hipSuccess)
        return fail(BBE_ENOMEM, "device allocation failed");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e =
        BBE_HIP(hipMemcpyAsync(d, h.data(), sizeof(bbe::ReqDesc) * n, hipMemcpyHostToDevice, s));
    if (e == hipSuccess)
        e = BBE_HIP(bbe::launch_prefix_batch(d, n, (uint32_t)seed, (uint32_t)(seed >> 32),
                                             tick_out, pos_out, prev_out, s));
    hipError_t e2 = hipStreamSynchronize(s);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(e, "in-play state batch");
    if (e2 != hipSuccess) return hip_fail(e2, "in-play state batch");
    return ok();
}

// ---------------------------------------------------------------------------
// bbe_prefix_batch without allocations: the request descriptors go to a
// fixed device array instead of a per-call hipMalloc.  The array exists once
// per GPU for the life of the process; host code reaches it only through
// the address hipGetSymbolAddress returns on that GPU (the array's own name
// is a host-side stand-in there).
// ---------------------------------------------------------------------------
static __device__ __align__(256) bbe::ReqDesc scratch[BBE_PREFIX_NOALLOC_MAX];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
bbe::ReqDesc* g_scratch_ptr[kMaxDevices] = {};

// Address of the current GPU's copy of `scratch`, looked up once per GPU
// with that GPU current.
int scratch_on_current_device(bbe::ReqDesc** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(BBE_EDEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "looking up the static workspace");
        g_scratch_ptr[dev] = static_cast<bbe::ReqDesc*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return BBE_OK;
}

}  // namespace

BBE_API int bbe_prefix_batch_noalloc(const bbe_request* reqs, const uint32_t* sims,
                                     const float* targets, int n, uint64_t seed,
                                     uint32_t* tick_out, float* pos_out, float* prev_out,
                                     void* stream) {
    if (!reqs || !sims || !targets || n < 1) return fail(BBE_EINVAL, "bad batch arguments");
    if (n > BBE_PREFIX_NOALLOC_MAX)
        return fail(BBE_EINVAL, "n = %d exceeds the static workspace of %d requests", n,
                    BBE_PREFIX_NOALLOC_MAX);
    if (!tick_out || !pos_out || !prev_out) return fail(BBE_EINVAL, "NULL output");
    bbe::ReqDesc* d = nullptr;
    int rc = scratch_on_current_device(&d);
    if (rc != BBE_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // descriptors staged through a fixed host block, one piece at a time
    constexpr int kPiece = 32;
    bbe::ReqDesc h[kPiece];
    for (int i0 = 0; i0 < n; i0 += kPiece) {
        const int m = std::min(kPiece, n - i0);
        for (int j = 0; j < m; ++j) {
            rc = fill_prefix_desc(reqs[i0 + j], sims[i0 + j], targets[i0 + j], i0 + j, h[j]);
            if (rc != BBE_OK) return rc;  // nothing launched yet; earlier pieces are unused
        }
        hipError_t e = BBE_HIP(hipMemcpyAsync(d + i0, h, sizeof(bbe::ReqDesc) * m,
                                              hipMemcpyHostToDevice, s));
        if (e == hipSuccess) e = hipStreamSynchronize(s);  // h is reused by the next piece
        if (e != hipSuccess) return hip_fail(e, "staging the request descriptors");
    }
    hipError_t e = BBE_HIP(bbe::launch_prefix_batch(d, n, (uint32_t)seed, (uint32_t)(seed >> 32),
                                                    tick_out, pos_out, prev_out, s));
    hipError_t e2 = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "in-play state batch");
    if (e2 != hipSuccess) return hip_fail(e2, "in-play state batch");
    return ok();
}
