// Batching extension: many uneven segments in one persistent launch (a
// device-side planner, a tile-parallel stage 1, a per-segment stage 2),
// stream capture into HIP graphs, and the autotuner.
//
// The autotuner follows the paper's automated tuning (section "Code
// Generation", "Automated Tuning": keep the variants, time them, choose at
// run time when complete information is available) and its future-work note
// on compiling the variants of a search on all CPU cores: candidates are
// generated and compiled concurrently through the same run-time compilation
// path, then timed with HIP events on the caller's data.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <functional>
#include <sstream>
#include <thread>

#include "internal.h"

using namespace hipmr;

struct hipmr_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace hipmr {

namespace {

constexpr int kSegBlock = 256, kSegIpt = 4, kSegBlocksPerCu = 8;
constexpr int kPlanBlock = 1024;
constexpr int kMaxLdsSegs = 8192;   // tile-start table in LDS up to this many entries

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// tiles of the smallest tile size any launch can use (one-element chunks,
// IPT = 1), so that every geometry and alignment fits the same workspace
long long max_tiles(int32_t nseg, int64_t total_n, int vec) {
    (void)vec;
    const long long t_min = 64;
    return (long long)nseg + (total_n + t_min - 1) / t_min + 1;
}

size_t seg_workspace(int32_t nseg, int64_t total_n, int vec) {
    return align256((size_t)(nseg + 1) * 4) + (size_t)max_tiles(nseg, total_n, vec) * 8;
}

std::string tune_key(const char* op, const char* combine, const char* neutral) {
    return std::string(op) + "\x1f" + (combine ? combine : "") + "\x1f" + (neutral ? neutral : "");
}

int lds_capacity(int32_t nseg) {
    if (nseg + 1 > kMaxLdsSegs) return 0;
    int cap = 256;
    while (cap < nseg + 1) cap *= 2;
    return cap;
}

struct SegLaunch {
    void* plan = nullptr;
    void* s1 = nullptr;
    void* s2 = nullptr;
    int grid1 = 0;
    long long head = 0;
    LaunchCfg cfg;
};

KernelSpec seg_spec(KernelKind kind, const LaunchCfg& cfg, bool idx64, const char* combine,
                    const char* neutral, int lds) {
    KernelSpec s;
    s.kind = kind;
    s.idx64 = idx64;
    s.block = kind == KernelKind::SegPlan ? kPlanBlock : cfg.block;
    s.ipt = cfg.ipt;
    s.vec = cfg.vec;
    s.nt_loads = cfg.nt_loads;
    s.nt_stores = cfg.nt_stores;
    if (kind != KernelKind::SegPlan) {
        s.combine = combine;
        s.neutral = neutral;
    }
    if (kind == KernelKind::SegS1) s.lds_segs = lds;
    if (kind == KernelKind::SegS2) {
        s.block = kSegBlock;
        s.ipt = 1;
        s.vec = 1;
        s.nt_loads = s.nt_stores = true;
    }
    if (kind == KernelKind::SegPlan) s.nt_loads = s.nt_stores = true;
    return s;
}

hipmr_status seg_prepare(hipmr_kernel* h, const char* combine, const char* neutral, int32_t nseg,
                         int64_t total_n, void* const* args, const LaunchCfg& cfg_in,
                         std::string* syms, SegLaunch* out) {
    LaunchCfg cfg = cfg_in;
    long long head = h->prog.info.vectorizable && !cfg.force_scalar ? common_head(h, args, cfg.vec) : -1;
    if (head < 0) {       // no common alignment (or scalar access): one-element chunks
        cfg.vec = 1;
        head = 0;
    }
    bool idx64 = total_n >= (int64_t(1) << 31);
    int lds = cfg.seg_global ? 0 : lds_capacity(nseg);
    hipmr_status st = HIPMR_OK;
    out->plan = nullptr;
    if (lds == 0) {       // the table does not fit LDS: a planning launch writes it to global memory
        st = variant_function(h, seg_spec(KernelKind::SegPlan, cfg, idx64, combine, neutral, lds),
                              &out->plan, syms);
        if (st != HIPMR_OK) return st;
    }
    st = variant_function(h, seg_spec(KernelKind::SegS1, cfg, idx64, combine, neutral, lds), &out->s1, syms);
    if (st != HIPMR_OK) return st;
    st = variant_function(h, seg_spec(KernelKind::SegS2, cfg, idx64, combine, neutral, lds), &out->s2, syms);
    if (st != HIPMR_OK) return st;
    long long tiles = max_tiles(nseg, total_n, cfg.vec);
    int waves_per_block = cfg.block / 64;
    int cap = (int)std::min<long long>((tiles + waves_per_block - 1) / waves_per_block, 1 << 20);
    out->grid1 = grid_for(cap, 1, cfg, std::max(cap, 1));
    out->head = head;
    out->cfg = cfg;
    return HIPMR_OK;
}

hipmr_status seg_launch(hipmr_kernel* h, const SegLaunch& L, int32_t nseg, const int64_t* d_offsets,
                        int64_t total_n, void* const* args, void* d_out, void* workspace,
                        void* stream) {
    void* tile_start = workspace;
    void* tpart = (char*)workspace + align256((size_t)(nseg + 1) * 4);
    long long total = total_n, head = L.head;
    // tile partials the workspace holds: the planner and both stages stop there
    long long cap = max_tiles(nseg, total_n, L.cfg.vec);
    const void* off = d_offsets;
    int ns = nseg;
    hipmr_status st = HIPMR_OK;
    if (L.plan) {
        void* p_plan[6] = {&off, &ns, &total, &head, &tile_start, &cap};
        st = launch(L.plan, 1, kPlanBlock, p_plan, stream);
        if (st != HIPMR_OK) return st;
    }
    std::vector<void*> p1;
    if (h->prog.sig.args.empty()) p1.push_back(&head);   // hipmr_unused
    for (size_t k = 0; k < h->prog.sig.args.size(); ++k) p1.push_back(args[k]);
    p1.push_back(&total);
    p1.push_back(&head);
    p1.push_back(&off);
    p1.push_back(&ns);
    p1.push_back(&tile_start);
    p1.push_back(&tpart);
    p1.push_back(&cap);
    st = launch(L.s1, (unsigned)L.grid1, (unsigned)L.cfg.block, p1.data(), stream);
    if (st != HIPMR_OK) return st;
    void* p2[5] = {&tile_start, &ns, &tpart, &d_out, &cap};
    unsigned grid2 = (unsigned)((nseg + kSegBlock / 64 - 1) / (kSegBlock / 64));
    return launch(L.s2, grid2, kSegBlock, p2, stream);
}

hipmr_status seg_checks(hipmr_kernel* h, const char* combine, const char* neutral, int32_t nseg,
                        const int64_t* d_offsets, int64_t total_n, void* const* args, void* d_out,
                        void* workspace, size_t ws_bytes) {
    hipmr_status st = check_args(h, total_n, args);
    if (st != HIPMR_OK) return st;
    if (!h->prog.sig.is_reduce) return fail(HIPMR_E_MISMATCH, "elementwise handle passed to a segmented reduce");
    if (!combine || !neutral) return fail(HIPMR_E_INVALID, "combine_op and neutral are required");
    if (nseg < 0) return fail(HIPMR_E_INVALID, "nseg must be >= 0");
    if (nseg > 0 && (!d_offsets || !d_out)) return fail(HIPMR_E_INVALID, "offsets or out is NULL");
    if (max_tiles(nseg, total_n, h->default_vec) > INT32_MAX)
        return fail(HIPMR_E_UNSUPPORTED, "segmented reduce: more than 2^31 - 1 tiles (total_n too large)");
    if (nseg > 0 && (!workspace || ws_bytes < seg_workspace(nseg, total_n, h->default_vec)))
        return fail(HIPMR_E_WORKSPACE, "workspace smaller than hipmr_segmented_workspace_bytes()");
    return HIPMR_OK;
}

// ------------------------------------------------------------ autotune store
std::string tune_dir() {
    const char* d = std::getenv("HIPMR_CACHE_DIR");
    std::string base;
    if (d && *d) base = d;
    else if (const char* x = std::getenv("XDG_CACHE_HOME"); x && *x) base = std::string(x) + "/hipmr";
    else base = std::string(std::getenv("HOME") ? std::getenv("HOME") : "/tmp") + "/.cache/hipmr";
    return base;
}

std::string tune_file(hipmr_kernel* h, const std::string& key, long long size_bucket) {
    std::string k = h->prog.name + "\x1f" + h->prog.expr + "\x1f" + key + "\x1f" +
                    std::to_string(size_bucket) + "\x1f" + std::to_string(h->prog.sig.args.size());
    for (auto& a : h->prog.sig.args) k += "\x1f" + std::to_string(a.dtype) + std::to_string(a.pointer);
    const char* arch = std::getenv("HIPMR_ARCH");
    k += std::string("\x1f") + (arch && *arch ? arch : "gfx950");
    return tune_dir() + "/tune_" + sha256_hex(k.data(), k.size()).substr(0, 32) + ".cfg";
}

bool load_tuned(hipmr_kernel* h, const std::string& key, long long bucket, hipmr_launch_config* out) {
    {
        std::lock_guard<std::mutex> lk(h->mu);
        auto it = h->tuned.find(key + "\x1f" + std::to_string(bucket));
        if (it != h->tuned.end()) {
            *out = it->second;
            return true;
        }
    }
    std::ifstream f(tune_file(h, key, bucket));
    hipmr_launch_config c{};
    if (!(f >> c.block >> c.items_per_thread >> c.grid >> c.blocks_per_cu >> c.vec >> c.flags)) return false;
    std::lock_guard<std::mutex> lk(h->mu);
    h->tuned[key + "\x1f" + std::to_string(bucket)] = c;
    *out = c;
    return true;
}

void store_tuned(hipmr_kernel* h, const std::string& key, long long bucket, const hipmr_launch_config& c) {
    {
        std::lock_guard<std::mutex> lk(h->mu);
        h->tuned[key + "\x1f" + std::to_string(bucket)] = c;
    }
    std::string path = tune_file(h, key, bucket);
    std::string tmp = path + ".tmp" + std::to_string((long long)std::hash<std::thread::id>()(std::this_thread::get_id()));
    {
        std::ofstream f(tmp);
        if (!f) return;
        f << c.block << " " << c.items_per_thread << " " << c.grid << " " << c.blocks_per_cu << " "
          << c.vec << " " << c.flags << "\n";
    }
    std::rename(tmp.c_str(), path.c_str());
}

long long bucket_of(long long n) {      // power-of-two size class
    long long b = 1;
    while (b < n) b <<= 1;
    return b;
}

// Candidate geometries for the autotuner.
std::vector<hipmr_launch_config> candidates(bool segmented) {
    std::vector<hipmr_launch_config> v;
    for (int block : {256, 512})
        for (int ipt : {1, 2, 4, 8})
            for (int bpc : segmented ? std::vector<int>{2, 4, 8, 16} : std::vector<int>{1, 2, 4, 8}) {
                hipmr_launch_config c{};
                c.block = block;
                c.items_per_thread = ipt;
                c.blocks_per_cu = bpc;
                v.push_back(c);
            }
    return v;
}

// Compiles the variants of every candidate concurrently (hipRTC programs are
// independent; the code-object cache is thread-safe).
hipmr_status compile_all(const std::vector<std::function<hipmr_status()>>& jobs) {
    std::atomic<size_t> next{0};
    std::atomic<int> status{HIPMR_OK};
    std::mutex err_mu;
    std::string err;
    unsigned nt = std::max(1u, std::min<unsigned>(std::thread::hardware_concurrency(), 16));
    std::vector<std::thread> pool;
    for (unsigned k = 0; k < nt; ++k)
        pool.emplace_back([&] {
            for (size_t j; (j = next++) < jobs.size();) {
                hipmr_status st = jobs[j]();
                if (st != HIPMR_OK) {
                    std::lock_guard<std::mutex> lk(err_mu);
                    if (status == HIPMR_OK) { status = st; err = last_error(); }
                }
            }
        });
    for (auto& t : pool) t.join();
    if (status != HIPMR_OK) return fail(status, err);
    return HIPMR_OK;
}

template <typename Run>
hipmr_status time_config(Run run, int reps, void* stream, float* ms) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
        return fail(HIPMR_E_HIP, "hipEventCreate failed");
    hipmr_status st = run();                          // warm-up (also loads the module)
    std::vector<float> t;
    for (int r = 0; r < reps && st == HIPMR_OK; ++r) {
        (void)hipEventRecord(a, (hipStream_t)stream);
        st = run();
        (void)hipEventRecord(b, (hipStream_t)stream);
        if (hipEventSynchronize(b) != hipSuccess) st = fail(HIPMR_E_HIP, "hipEventSynchronize failed");
        float x = 0;
        (void)hipEventElapsedTime(&x, a, b);
        t.push_back(x);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st != HIPMR_OK) return st;
    std::sort(t.begin(), t.end());
    *ms = t.empty() ? 0.f : t[t.size() / 2];
    return HIPMR_OK;
}

thread_local bool g_capturing = false;
thread_local bool g_no_alloc = false;

}  // namespace

bool capturing_now() { return g_capturing; }
bool no_alloc_now() { return g_no_alloc; }
void set_no_alloc(bool on) { g_no_alloc = on; }

size_t segmented_workspace(const hipmr_kernel* h, int32_t nseg, int64_t total_n) {
    return seg_workspace(nseg, total_n, h->default_vec);
}

hipmr_status reduce_segmented_on(hipmr_kernel* h, const char* combine, const char* neutral,
                                 int32_t nseg, const int64_t* d_offsets, int64_t total_n,
                                 void* const* args, void* d_out, void* workspace,
                                 size_t workspace_bytes, const hipmr_launch_config* cfgp,
                                 void* stream) {
    hipmr_status st = seg_checks(h, combine, neutral, nseg, d_offsets, total_n, args, d_out, workspace,
                                 workspace_bytes);
    if (st != HIPMR_OK) return st;
    if (nseg == 0) return HIPMR_OK;
    hipmr_launch_config tuned{};
    cfgp = apply_tuned(h, "seg", combine, neutral, total_n, cfgp, &tuned);
    LaunchCfg cfg;
    st = resolve_cfg(cfgp, kSegBlock, kSegIpt, h->default_vec, kSegBlocksPerCu, &cfg);
    if (st != HIPMR_OK) return st;
    std::string syms;
    SegLaunch L;
    st = seg_prepare(h, combine, neutral, nseg, total_n, args, cfg, &syms, &L);
    if (st != HIPMR_OK) return st;
    set_last_symbols(h, syms);
    return seg_launch(h, L, nseg, d_offsets, total_n, args, d_out, workspace, stream);
}

bool tuned_config(hipmr_kernel* h, const char* op, const char* combine, const char* neutral,
                  long long n, hipmr_launch_config* out) {
    return load_tuned(h, tune_key(op, combine, neutral), bucket_of(n), out);
}

const hipmr_launch_config* apply_tuned(hipmr_kernel* h, const char* op, const char* combine,
                                       const char* neutral, long long n,
                                       const hipmr_launch_config* cfgp, hipmr_launch_config* buf) {
    if (!cfgp || !(cfgp->flags & HIPMR_CFG_TUNED)) return cfgp;
    *buf = *cfgp;
    buf->flags &= ~HIPMR_CFG_TUNED;
    hipmr_launch_config t{};
    LaunchCfg probe;
    // a stored geometry that no longer resolves (an edited or stale file) is
    // ignored: the caller's geometry applies
    if (tuned_config(h, op, combine, neutral, n, &t) &&
        resolve_cfg(&t, 256, 1, 1, 1, &probe) == HIPMR_OK) {
        t.flags &= ~HIPMR_CFG_TUNED;
        *buf = t;
    }
    clear_error();
    return buf;
}

}  // namespace hipmr

extern "C" {

size_t hipmr_segmented_workspace_bytes(hipmr_handle h, int32_t nseg, int64_t total_n) {
    if (!h || !h->prog.sig.is_reduce || nseg < 0 || total_n < 0) return 0;
    return seg_workspace(nseg, total_n, h->default_vec);
}

hipmr_status hipmr_reduce_segmented(hipmr_handle h, const char* combine, const char* neutral,
                                    int32_t nseg, const int64_t* d_offsets, int64_t total_n,
                                    void* const* args, void* d_out, void* workspace,
                                    size_t workspace_bytes, const hipmr_launch_config* cfgp,
                                    void* stream) {
    clear_error();
    return reduce_segmented_on(h, combine, neutral, nseg, d_offsets, total_n, args, d_out, workspace,
                               workspace_bytes, cfgp, stream);
}

hipmr_status hipmr_autotune_segmented(hipmr_handle h, const char* combine, const char* neutral,
                                      int32_t nseg, const int64_t* d_offsets, int64_t total_n,
                                      void* const* args, void* d_out, void* workspace,
                                      size_t workspace_bytes, int32_t reps,
                                      hipmr_launch_config* best, void* stream) {
    clear_error();
    hipmr_status st = seg_checks(h, combine, neutral, nseg, d_offsets, total_n, args, d_out, workspace,
                                 workspace_bytes);
    if (st != HIPMR_OK) return st;
    if (nseg == 0 || reps < 1) return fail(HIPMR_E_INVALID, "autotuning needs nseg > 0 and reps >= 1");
    auto cands = candidates(true);
    std::vector<std::function<hipmr_status()>> jobs;
    std::vector<SegLaunch> plans(cands.size());
    for (size_t c = 0; c < cands.size(); ++c)
        jobs.push_back([&, c] {
            LaunchCfg cfg;
            hipmr_status s2 = resolve_cfg(&cands[c], kSegBlock, kSegIpt, h->default_vec, kSegBlocksPerCu, &cfg);
            if (s2 != HIPMR_OK) return s2;
            // compile only: building variants never touches the GPU
            long long head = h->prog.info.vectorizable ? common_head(h, args, cfg.vec) : -1;
            if (head < 0) cfg.vec = 1;
            bool idx64 = total_n >= (int64_t(1) << 31);
            int lds = lds_capacity(nseg);
            std::shared_ptr<CodeObject> co;
            for (KernelKind k : {KernelKind::SegPlan, KernelKind::SegS1, KernelKind::SegS2}) {
                s2 = get_variant(h, seg_spec(k, cfg, idx64, combine, neutral, lds), &co);
                if (s2 != HIPMR_OK) return s2;
            }
            return HIPMR_OK;
        });
    st = compile_all(jobs);
    if (st != HIPMR_OK) return st;
    float best_ms = 1e30f;
    hipmr_launch_config best_cfg{};
    for (size_t c = 0; c < cands.size(); ++c) {
        LaunchCfg cfg;
        st = resolve_cfg(&cands[c], kSegBlock, kSegIpt, h->default_vec, kSegBlocksPerCu, &cfg);
        if (st != HIPMR_OK) return st;
        std::string syms;
        SegLaunch L;
        st = seg_prepare(h, combine, neutral, nseg, total_n, args, cfg, &syms, &L);
        if (st != HIPMR_OK) return st;
        float ms = 0;
        st = time_config([&] { return seg_launch(h, L, nseg, d_offsets, total_n, args, d_out, workspace, stream); },
                         reps, stream, &ms);
        if (st != HIPMR_OK) return st;
        if (ms < best_ms) {
            best_ms = ms;
            best_cfg = cands[c];
        }
    }
    store_tuned(h, tune_key("seg", combine, neutral), bucket_of(total_n), best_cfg);
    if (best) *best = best_cfg;
    return HIPMR_OK;
}

hipmr_status hipmr_autotune_reduce(hipmr_handle h, const char* combine, const char* neutral, int64_t n,
                                   void* const* args, void* out, void* workspace,
                                   size_t workspace_bytes, int32_t reps, hipmr_launch_config* best,
                                   void* stream) {
    clear_error();
    hipmr_status st = check_args(h, n, args);
    if (st != HIPMR_OK) return st;
    if (!h->prog.sig.is_reduce) return fail(HIPMR_E_MISMATCH, "elementwise handle passed to hipmr_autotune_reduce");
    if (!combine || !neutral || !out) return fail(HIPMR_E_INVALID, "NULL argument");
    if (n <= 0 || reps < 1) return fail(HIPMR_E_INVALID, "autotuning needs n > 0 and reps >= 1");
    auto cands = candidates(false);
    std::vector<std::function<hipmr_status()>> jobs;
    for (size_t c = 0; c < cands.size(); ++c)
        jobs.push_back([&, c] {
            // building the stage-1 variant of each candidate concurrently
            hipmr_launch_config cc = cands[c];
            cc.grid = 0;
            return hipmr_prepare_reduce_ex(h, combine, neutral, &cc);
        });
    st = compile_all(jobs);
    if (st != HIPMR_OK) return st;
    float best_ms = 1e30f;
    hipmr_launch_config best_cfg{};
    for (auto& c : cands) {
        float ms = 0;
        st = time_config([&] {
            return hipmr_reduce_ex(h, nullptr, combine, neutral, n, args, out, workspace, workspace_bytes, &c, stream);
        }, reps, stream, &ms);
        if (st != HIPMR_OK) return st;
        if (ms < best_ms) {
            best_ms = ms;
            best_cfg = c;
        }
    }
    store_tuned(h, tune_key("reduce", combine, neutral), bucket_of(n), best_cfg);
    if (best) *best = best_cfg;
    return HIPMR_OK;
}

hipmr_status hipmr_graph_begin_capture(void* stream) {
    clear_error();
    if (!stream) return fail(HIPMR_E_INVALID, "the null stream cannot be captured");
    hipError_t e = hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail(HIPMR_E_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    g_capturing = true;
    return HIPMR_OK;
}

hipmr_status hipmr_graph_end_capture(void* stream, hipmr_graph_t* out) {
    clear_error();
    g_capturing = false;
    if (!stream || !out) return fail(HIPMR_E_INVALID, "NULL argument");
    auto g = std::make_unique<hipmr_graph>();
    hipError_t e = hipStreamEndCapture((hipStream_t)stream, &g->graph);
    if (e != hipSuccess) return fail(HIPMR_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g->graph);
        return fail(HIPMR_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    *out = g.release();
    return HIPMR_OK;
}

hipmr_status hipmr_graph_launch(hipmr_graph_t g, void* stream) {
    clear_error();
    if (!g) return fail(HIPMR_E_INVALID, "NULL graph");
    hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    if (e != hipSuccess) return fail(HIPMR_E_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    return HIPMR_OK;
}

void hipmr_graph_destroy(hipmr_graph_t g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

}  // extern "C"
