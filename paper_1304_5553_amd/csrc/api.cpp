// The C ABI: handles, argument marshalling, launch geometry and the two
// launch sequences (elementwise; map-reduce = block partials + final fold).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <cctype>
#include <cstring>
#include <map>
#include <memory>
#include <unordered_map>

#include "internal.h"

using namespace hipmr;

namespace hipmr {

int default_vec_for(const Signature& sig) {
    int min_size = 0;
    for (auto& a : sig.args)
        if (chunked(a) || a.shifted) {
            int s = dtype_size(a.dtype);
            if (min_size == 0 || s < min_size) min_size = s;
        }
    if (min_size == 0) return 4;
    return 16 / min_size;
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

hipmr_status resolve_cfg(const hipmr_launch_config* c, int block, int ipt, int vec,
                         int blocks_per_cu, LaunchCfg* out) {
    *out = LaunchCfg();
    out->block = block;
    out->ipt = ipt;
    out->vec = vec;
    out->blocks_per_cu = blocks_per_cu;
    if (!c) return HIPMR_OK;
    if (c->block) {
        if (c->block < 64 || c->block > 1024 || c->block % 64)
            return fail(HIPMR_E_INVALID, "launch config: block must be a multiple of 64 in [64, 1024]");
        out->block = c->block;
    }
    if (c->items_per_thread) {
        if (c->items_per_thread < 1 || c->items_per_thread > 16)
            return fail(HIPMR_E_INVALID, "launch config: items_per_thread must be in [1, 16]");
        out->ipt = c->items_per_thread;
    }
    if (c->vec) {
        if (!is_pow2(c->vec) || c->vec > 16)
            return fail(HIPMR_E_INVALID, "launch config: vec must be a power of two <= 16");
        out->vec = c->vec;
    }
    if (c->grid < 0 || c->blocks_per_cu < 0)
        return fail(HIPMR_E_INVALID, "launch config: negative grid or blocks_per_cu");
    out->grid = c->grid;
    if (c->blocks_per_cu) out->blocks_per_cu = c->blocks_per_cu;
    if (c->flags & HIPMR_CFG_TEMPORAL) out->nt_loads = out->nt_stores = false;
    if (c->flags & HIPMR_CFG_NONTEMPORAL) out->nt_loads = out->nt_stores = true;
    if (c->flags & HIPMR_CFG_TEMPORAL_LOADS) out->nt_loads = false;
    if (c->flags & HIPMR_CFG_TEMPORAL_STORES) out->nt_stores = false;
    out->force_scalar = (c->flags & HIPMR_CFG_FORCE_SCALAR) != 0;
    out->seg_global = (c->flags & HIPMR_CFG_SEG_GLOBAL) != 0;
    return HIPMR_OK;
}

std::string spec_key(const KernelSpec& s) {
    return std::to_string((int)s.kind) + "|" + std::to_string(s.idx64) + "|" +
           std::to_string(s.block) + "|" + std::to_string(s.ipt) + "|" + std::to_string(s.vec) +
           "|" + std::to_string(s.nt_loads) + std::to_string(s.nt_stores) + "|" +
           std::to_string(s.square) + std::to_string(s.scaled) + std::to_string(s.exact_runs) +
           std::to_string(s.norm) + "|" + std::to_string(s.lds_segs) + "|" + s.combine + "\x1f" +
           s.neutral;
}

hipmr_status get_variant(hipmr_kernel* h, const KernelSpec& spec, std::shared_ptr<CodeObject>* out) {
    if (h->prog.sig.result == DT_C64 && !spec.combine.empty() &&
        canonical_combine(spec.combine) != Combine::Sum && canonical_combine(spec.combine) != Combine::Generic)
        return fail(HIPMR_E_UNSUPPORTED, "complex values have no order: reduce them with a sum");
    std::string k = spec_key(spec);
    {
        std::lock_guard<std::mutex> lk(h->mu);
        auto it = h->variants.find(k);
        if (it != h->variants.end()) {
            *out = it->second;
            return HIPMR_OK;
        }
    }
    if (no_alloc_now())
        return fail(HIPMR_E_INVALID, "this kernel variant has not been built for the handle: run the "
                                     "allocating entry point once with the same arguments first");
    std::string symbol;
    std::string src = render(h->prog, spec, &symbol);
    hipmr_status st;
    auto co = get_or_build(src, symbol, &st);
    if (!co) return st;
    std::lock_guard<std::mutex> lk(h->mu);
    h->variants[k] = co;
    *out = co;
    return HIPMR_OK;
}

// Function of a variant on the current device; appends its symbol to *syms.
hipmr_status variant_function(hipmr_kernel* h, const KernelSpec& spec, void** fn,
                              std::string* syms) {
    std::shared_ptr<CodeObject> co;
    hipmr_status st = get_variant(h, spec, &co);
    if (st != HIPMR_OK) return st;
    if (syms) *syms += (syms->empty() ? "" : ",") + code_object_symbol(*co);
    return get_function(*co, fn);
}

void set_last_symbols(hipmr_kernel* h, const std::string& syms) {
    std::lock_guard<std::mutex> lk(h->mu);
    h->last_symbols = syms;
}

// Element offset "head" at which every accessed array is aligned for the
// vector chunk loads; -1 if no common offset exists.
long long common_head(const hipmr_kernel* h, void* const* args, int vec) {
    for (int head = 0; head < vec; ++head) {
        bool ok = true;
        for (size_t k = 0; k < h->prog.sig.args.size() && ok; ++k) {
            const ArgDecl& a = h->prog.sig.args[k];
            if (!chunked(a)) continue;
            uintptr_t p = (uintptr_t)(*(void* const*)args[k]);
            int s = dtype_size(a.dtype);
            uintptr_t align = (uintptr_t)std::min(vec * s, 16);
            if (p % (uintptr_t)s != 0 || (p + (uintptr_t)head * s) % align != 0) ok = false;
        }
        if (ok) return head;
    }
    return -1;
}

hipmr_status check_args(hipmr_kernel* h, int64_t n, void* const* args) {
    if (!h) return fail(HIPMR_E_INVALID, "NULL handle");
    if (n < 0) return fail(HIPMR_E_INVALID, "n must be >= 0");
    const auto& decl = h->prog.sig.args;
    if (!decl.empty() && !args) return fail(HIPMR_E_INVALID, "args is NULL");
    for (size_t k = 0; k < decl.size(); ++k) {
        if (!args[k]) return fail(HIPMR_E_INVALID, "args[" + std::to_string(k) + "] is NULL");
        if (decl[k].pointer && n > 0 && (decl[k].read || decl[k].written) &&
            *(void* const*)args[k] == nullptr)
            return fail(HIPMR_E_INVALID, "array argument '" + decl[k].name + "' is NULL");
    }
    return HIPMR_OK;
}

int grid_for(long long work_units, int per_block, const LaunchCfg& cfg, int cap) {
    cap = (int)std::min<long long>(cap, ((1LL << 32) - 1) / cfg.block);   // threads < 2^32
    if (cfg.grid > 0) return std::min(cfg.grid, cap);
    long long need = (work_units + per_block - 1) / per_block;
    long long limit = (long long)cfg.blocks_per_cu * device_cu_count();
    long long g = std::min(need, limit);
    g = std::min<long long>(g, cap);
    return (int)std::max<long long>(g, 1);
}

// Handles are cached by (name, dtypes, expr) as given: compiling the same
// text again returns the same handle with one more reference, which costs a
// hash lookup (section "Core Method": kernels already built are reused
// instead of being generated again).  The last hipmr_release removes the
// handle from the cache and frees it.  All reference counting happens under
// g_handles_mu, so a lookup never revives a handle that is being freed.
std::mutex g_handles_mu;
std::unordered_map<std::string, hipmr_kernel*> g_handles;

std::string handle_key(const char* expr, const char* dtypes, const std::string& name) {
    std::string k;
    k.reserve(name.size() + std::strlen(dtypes) + std::strlen(expr) + 2);
    k += name;
    k += '\x1f';
    k += dtypes;
    k += '\x1f';
    k += expr;
    return k;
}

hipmr_status build_handle(const char* expr, const char* dtypes, const std::string& nm,
                          std::unique_ptr<hipmr_kernel>* out);

hipmr_status make_handle(const char* expr, const char* dtypes, const char* name,
                         hipmr_handle* out) {
    if (!expr || !dtypes || !out) return fail(HIPMR_E_INVALID, "NULL argument to hipmr_compile");
    *out = nullptr;
    std::string nm = name && *name ? name : "hipmr";
    std::string key = handle_key(expr, dtypes, nm);
    {
        std::lock_guard<std::mutex> lk(g_handles_mu);
        auto it = g_handles.find(key);
        if (it != g_handles.end()) {
            ++it->second->refs;
            *out = it->second;
            return HIPMR_OK;
        }
    }
    std::unique_ptr<hipmr_kernel> h;
    hipmr_status st = build_handle(expr, dtypes, nm, &h);      // front end, codegen, compile
    if (st != HIPMR_OK) return st;
    std::lock_guard<std::mutex> lk(g_handles_mu);
    auto ins = g_handles.emplace(key, h.get());
    if (!ins.second) {                 // another thread built the same handle meanwhile
        ++ins.first->second->refs;
        *out = ins.first->second;
        return HIPMR_OK;
    }
    h->cache_key = key;
    h->cached = true;
    *out = h.release();
    return HIPMR_OK;
}

void release_handle(hipmr_kernel* h) {
    {
        std::lock_guard<std::mutex> lk(g_handles_mu);
        if (--h->refs > 0) return;
        if (h->cached) {
            auto it = g_handles.find(h->cache_key);
            if (it != g_handles.end() && it->second == h) g_handles.erase(it);
        }
    }
    delete h;
}

// Forgets the cached handles (they stay valid for their holders, who free
// them with their last release); compile() then builds new ones.
void drop_handle_cache() {
    std::lock_guard<std::mutex> lk(g_handles_mu);
    for (auto& kv : g_handles) kv.second->cached = false;
    g_handles.clear();
}

hipmr_status build_handle(const char* expr, const char* dtypes, const std::string& nm,
                          std::unique_ptr<hipmr_kernel>* out) {
    for (char c : nm)
        if (!(std::isalnum((unsigned char)c) || c == '_'))
            return fail(HIPMR_E_INVALID, "kernel name must be a C identifier");
    auto h = std::make_unique<hipmr_kernel>();
    h->refs = 1;
    h->prog.name = nm;
    h->prog.expr = expr;
    hipmr_status st = parse_signature(dtypes, &h->prog.sig);
    if (st != HIPMR_OK) return st;
    st = lex(expr, &h->prog.toks);
    if (st != HIPMR_OK) return st;
    if (h->prog.toks.size() <= 1) return fail(HIPMR_E_PARSE, "empty expression");
    st = classify(h->prog.toks, &h->prog.sig, h->prog.sig.is_reduce, &h->prog.info);
    if (st != HIPMR_OK) return st;
    if (h->prog.sig.is_reduce) {
        DType r = h->prog.sig.result;
        if (!(r == DT_F32 || r == DT_F64 || r == DT_I32 || r == DT_U32 || r == DT_I64 || r == DT_C64))
            return fail(HIPMR_E_UNSUPPORTED, "reduce result type must be float, double, int, "
                                             "unsigned, a 64-bit integer or complex64");
    }
    h->default_vec = default_vec_for(h->prog.sig);
    if (!h->prog.sig.is_reduce) {
        // build the default variant now so that errors surface at compile time
        KernelSpec spec;
        spec.kind = h->prog.info.vectorizable ? KernelKind::EwVector : KernelKind::EwScalar;
        spec.block = kEwBlock;
        spec.ipt = kEwIpt;
        spec.vec = h->default_vec;
        std::shared_ptr<CodeObject> co;
        st = get_variant(h.get(), spec, &co);
        if (st != HIPMR_OK) return st;
    }
    *out = std::move(h);
    return HIPMR_OK;
}

KernelSpec s1_spec(const hipmr_kernel* h, bool vector, const LaunchCfg& cfg, bool idx64,
                   const char* combine, const char* neutral) {
    KernelSpec s;
    s.kind = vector ? KernelKind::RedS1Vector : KernelKind::RedS1Scalar;
    s.idx64 = idx64;
    s.block = cfg.block;
    s.ipt = cfg.ipt;
    s.vec = vector ? cfg.vec : 1;
    s.nt_loads = cfg.nt_loads;
    s.nt_stores = cfg.nt_stores;
    s.combine = combine;
    s.neutral = neutral;
    return s;
}

KernelSpec s2_spec(const char* combine, const char* neutral) {
    KernelSpec s;
    s.kind = KernelKind::RedS2;
    s.block = kStage2Block;
    s.ipt = 1;
    s.vec = 1;
    s.combine = combine;
    s.neutral = neutral;
    return s;
}

}  // namespace hipmr


namespace {

// Shared launch logic of the precision extension: one stage-1 kernel over the
// map (vector when possible), its partials, and one finishing kernel.
struct Stage1 {
    void* fn = nullptr;
    int grid = 0;
    long long head = 0;
};

hipmr_status stage1_launch(hipmr_kernel* h, KernelSpec spec, bool vector_ok, const LaunchCfg& cfg,
                           int64_t n, void* const* args, void* partial, void* extra,
                           bool with_extra, void* stream, std::string* syms, Stage1* out) {
    long long head = -1;
    bool vector = vector_ok && h->prog.info.vectorizable && !cfg.force_scalar;
    if (vector) head = common_head(h, args, cfg.vec);
    if (head < 0) vector = false;
    if (!vector) {
        switch (spec.kind) {
            case KernelKind::CompS1Vector: spec.kind = KernelKind::CompS1Scalar; break;
            case KernelKind::AmaxS1Vector: spec.kind = KernelKind::AmaxS1Scalar; break;
            default: break;
        }
        spec.vec = 1;
        spec.exact_runs = false;
    }
    spec.idx64 = n >= (int64_t(1) << 31);
    hipmr_status st = variant_function(h, spec, &out->fn, syms);
    if (st != HIPMR_OK) return st;
    long long n64 = n, head64 = vector ? head : 0;
    long long units = vector ? (n64 > head64 ? (n64 - head64) / cfg.vec : 0) : n64;
    out->grid = n > 0 ? grid_for(units, cfg.block * (vector ? cfg.ipt : 1), cfg, kMaxPartials) : 0;
    out->head = head64;
    if (n == 0) return HIPMR_OK;
    std::vector<void*> params;
    if (h->prog.sig.args.empty()) params.push_back(&head64);   // hipmr_unused
    for (size_t k = 0; k < h->prog.sig.args.size(); ++k) params.push_back(args[k]);
    params.push_back(&n64);
    params.push_back(&head64);
    params.push_back(&partial);
    if (with_extra) params.push_back(&extra);
    return launch(out->fn, (unsigned)out->grid, (unsigned)cfg.block, params.data(), stream);
}

KernelSpec comp_spec(KernelKind kind, const LaunchCfg& cfg) {
    KernelSpec s;
    s.kind = kind;
    s.block = cfg.block;
    s.ipt = cfg.ipt;
    s.vec = cfg.vec;
    s.nt_loads = cfg.nt_loads;
    s.nt_stores = cfg.nt_stores;
    return s;
}

// The map is a single load of an FP8 array: runs of <= 64 values sum exactly.
bool single_fp8_load(const hipmr_kernel* h) {
    const auto& t = h->prog.toks;
    if (t.size() != 5 || t[0].kind != Token::Ident || t[1].text != "[" || t[2].text != "i" ||
        t[3].text != "]")
        return false;
    for (const ArgDecl& a : h->prog.sig.args)
        if (a.name == t[0].text) return a.pointer && a.dtype == DT_FP8;
    return false;
}

hipmr_status precision_checks(hipmr_kernel* h, int64_t n, void* const* args, void* out,
                              void* workspace, size_t workspace_bytes) {
    hipmr_status st = check_args(h, n, args);
    if (st != HIPMR_OK) return st;
    if (!h->prog.sig.is_reduce || h->prog.sig.result != DT_F32)
        return fail(HIPMR_E_MISMATCH, "the precision extension needs a 'float:' map-reduce handle "
                                      "(the map is accumulated in compensated float)");
    if (!out) return fail(HIPMR_E_INVALID, "out is NULL");
    if (!workspace || workspace_bytes < kWorkspaceBytes)
        return fail(HIPMR_E_WORKSPACE, "workspace smaller than hipmr_reduce_workspace_bytes()");
    return HIPMR_OK;
}

}  // namespace

extern "C" {

hipmr_status hipmr_reduce_compensated(hipmr_handle h, int64_t n, void* const* args,
                                      double post_scale, void* out, void* workspace,
                                      size_t workspace_bytes, const hipmr_launch_config* cfgp,
                                      void* stream) {
    clear_error();
    hipmr_status st = precision_checks(h, n, args, out, workspace, workspace_bytes);
    if (st != HIPMR_OK) return st;
    LaunchCfg cfg;
    st = resolve_cfg(cfgp, kRedBlock, kRedIpt, h->default_vec, kRedBlocksPerCu, &cfg);
    if (st != HIPMR_OK) return st;
    KernelSpec s1 = comp_spec(KernelKind::CompS1Vector, cfg);
    s1.exact_runs = single_fp8_load(h) && cfg.vec * cfg.ipt <= 64;
    std::string syms;
    Stage1 r;
    st = stage1_launch(h, s1, true, cfg, n, args, workspace, nullptr, true, stream, &syms, &r);
    if (st != HIPMR_OK) return st;
    KernelSpec s2 = comp_spec(KernelKind::CompS2, cfg);
    s2.block = kStage2Block;
    s2.ipt = s2.vec = 1;
    void* fn2 = nullptr;
    st = variant_function(h, s2, &fn2, &syms);
    if (st != HIPMR_OK) return st;
    set_last_symbols(h, syms);
    void* scale64 = (char*)workspace + kScaleOffset + 8;
    void* params2[5] = {&workspace, &r.grid, &post_scale, &scale64, &out};
    return launch(fn2, 1, kStage2Block, params2, stream);
}

hipmr_status hipmr_norm2(hipmr_handle h, int64_t n, void* const* args, double post_scale,
                         int32_t passes, void* out, void* workspace, size_t workspace_bytes,
                         const hipmr_launch_config* cfgp, void* stream) {
    clear_error();
    hipmr_status st = precision_checks(h, n, args, out, workspace, workspace_bytes);
    if (st != HIPMR_OK) return st;
    if (passes != 1 && passes != 2) return fail(HIPMR_E_INVALID, "passes must be 1 or 2");
    LaunchCfg cfg;
    st = resolve_cfg(cfgp, kRedBlock, kRedIpt, h->default_vec, kRedBlocksPerCu, &cfg);
    if (st != HIPMR_OK) return st;
    void* amax = (char*)workspace + kAmaxOffset;
    void* scale_d = (char*)workspace + kScaleOffset + 8;
    std::string syms;
    const bool two = passes == 2 && n > 0;     // an empty norm is 0 either way
    if (two) {
        // pass 1: exact max |map| per block (the same grid as pass 2)
        KernelSpec a1 = comp_spec(KernelKind::AmaxS1Vector, cfg);
        Stage1 r1;
        st = stage1_launch(h, a1, true, cfg, n, args, amax, nullptr, false, stream, &syms, &r1);
        if (st != HIPMR_OK) return st;
    }
    // pass 2 (or the only pass): compensated sum of (map * scale)^2; with two
    // passes every block first derives the power-of-two scale from the pass-1
    // partials (block 0 also stores it for the final fold)
    KernelSpec q1 = comp_spec(KernelKind::CompS1Vector, cfg);
    q1.square = true;
    q1.scaled = two;
    Stage1 r2;
    st = stage1_launch(h, q1, true, cfg, n, args, workspace, amax, true, stream, &syms, &r2);
    if (st != HIPMR_OK) return st;
    KernelSpec q2 = comp_spec(KernelKind::CompS2, cfg);
    q2.block = kStage2Block;
    q2.ipt = q2.vec = 1;
    q2.norm = true;
    q2.scaled = two;
    void* fn2 = nullptr;
    st = variant_function(h, q2, &fn2, &syms);
    if (st != HIPMR_OK) return st;
    set_last_symbols(h, syms);
    void* params2[5] = {&workspace, &r2.grid, &post_scale, &scale_d, &out};
    return launch(fn2, 1, kStage2Block, params2, stream);
}

}  // extern "C"

extern "C" {

hipmr_status hipmr_compile(const char* expr, const char* dtypes, hipmr_handle* out) {
    clear_error();
    return make_handle(expr, dtypes, nullptr, out);
}

hipmr_status hipmr_compile_named(const char* expr, const char* dtypes, const char* name,
                                 hipmr_handle* out) {
    clear_error();
    return make_handle(expr, dtypes, name, out);
}

hipmr_status hipmr_elementwise_ex(hipmr_handle h, int64_t n, void* const* args,
                                  const hipmr_launch_config* cfgp, void* stream) {
    clear_error();
    hipmr_status st = check_args(h, n, args);
    if (st != HIPMR_OK) return st;
    if (h->prog.sig.is_reduce) return fail(HIPMR_E_MISMATCH, "map-reduce handle passed to hipmr_elementwise");
    LaunchCfg cfg;
    st = resolve_cfg(cfgp, kEwBlock, kEwIpt, h->default_vec, kEwBlocksPerCu, &cfg);
    if (st != HIPMR_OK) return st;
    if (n == 0) return HIPMR_OK;
    long long head = -1;
    bool vector = h->prog.info.vectorizable && !cfg.force_scalar;
    if (vector) head = common_head(h, args, cfg.vec);
    if (head < 0) vector = false;
    // the one-element kernel does best as a grid-stride loop over a resident
    // grid (measured on MI355X with a five-point stencil: 30 us against 37 us
    // for one element per thread over a full grid)
    if (!vector && !(cfgp && (cfgp->blocks_per_cu || cfgp->grid))) cfg.blocks_per_cu = kEwScalarBlocksPerCu;
    KernelSpec spec;
    spec.kind = vector ? KernelKind::EwVector : KernelKind::EwScalar;
    spec.idx64 = n >= (int64_t(1) << 31);
    spec.block = cfg.block;
    spec.ipt = cfg.ipt;
    spec.vec = vector ? cfg.vec : 1;
    spec.nt_loads = cfg.nt_loads;
    spec.nt_stores = cfg.nt_stores;
    void* fn = nullptr;
    std::string syms;
    st = variant_function(h, spec, &fn, &syms);
    if (st != HIPMR_OK) return st;
    set_last_symbols(h, syms);
    long long n64 = n, head64 = vector ? head : 0;
    long long units = vector ? (n64 > head64 ? (n64 - head64) / cfg.vec : 0) : n64;
    int grid = grid_for(units, cfg.block * (vector ? cfg.ipt : 1), cfg, 1 << 30);
    std::vector<void*> params;
    if (h->prog.sig.args.empty()) params.push_back(&head64);   // hipmr_unused
    for (size_t k = 0; k < h->prog.sig.args.size(); ++k) params.push_back(args[k]);
    params.push_back(&n64);
    params.push_back(&head64);
    return launch(fn, (unsigned)grid, (unsigned)cfg.block, params.data(), stream);
}

hipmr_status hipmr_elementwise(hipmr_handle h, int64_t n, void* const* args, void* stream) {
    return hipmr_elementwise_ex(h, n, args, nullptr, stream);
}

size_t hipmr_reduce_workspace_bytes(hipmr_handle h, int64_t n) {
    (void)n;
    if (!h || !h->prog.sig.is_reduce) return 0;
    return kWorkspaceBytes;
}

hipmr_status hipmr_prepare_reduce_ex(hipmr_handle h, const char* combine, const char* neutral,
                                     const hipmr_launch_config* cfgp) {
    clear_error();
    if (!h || !combine || !neutral) return fail(HIPMR_E_INVALID, "NULL argument");
    if (!h->prog.sig.is_reduce) return fail(HIPMR_E_MISMATCH, "elementwise handle");
    LaunchCfg cfg;
    hipmr_status rs = resolve_cfg(cfgp, kRedBlock, kRedIpt, h->default_vec, kRedBlocksPerCu, &cfg);
    if (rs != HIPMR_OK) return rs;
    std::shared_ptr<CodeObject> co;
    hipmr_status st = get_variant(h, s1_spec(h, h->prog.info.vectorizable, cfg, false, combine, neutral), &co);
    if (st != HIPMR_OK) return st;
    return get_variant(h, s2_spec(combine, neutral), &co);
}

hipmr_status hipmr_prepare_reduce(hipmr_handle h, const char* combine, const char* neutral) {
    return hipmr_prepare_reduce_ex(h, combine, neutral, nullptr);
}

hipmr_status hipmr_reduce_ex(hipmr_handle h, const char* map_expr, const char* combine,
                             const char* neutral, int64_t n, void* const* args, void* out,
                             void* workspace, size_t workspace_bytes,
                             const hipmr_launch_config* cfgp, void* stream) {
    clear_error();
    hipmr_status st = check_args(h, n, args);
    if (st != HIPMR_OK) return st;
    if (!h->prog.sig.is_reduce) return fail(HIPMR_E_MISMATCH, "elementwise handle passed to hipmr_reduce");
    if (map_expr && h->prog.expr != map_expr)
        return fail(HIPMR_E_MISMATCH, "map_expr differs from the handle's expression");
    if (!combine || !neutral) return fail(HIPMR_E_INVALID, "combine_op and neutral are required");
    if (!out) return fail(HIPMR_E_INVALID, "out is NULL");
    if (!workspace || workspace_bytes < hipmr_reduce_workspace_bytes(h, n))
        return fail(HIPMR_E_WORKSPACE, "workspace smaller than hipmr_reduce_workspace_bytes()");
    hipmr_launch_config tuned{};
    cfgp = apply_tuned(h, "reduce", combine, neutral, n, cfgp, &tuned);
    LaunchCfg cfg;
    st = resolve_cfg(cfgp, kRedBlock, kRedIpt, h->default_vec, kRedBlocksPerCu, &cfg);
    if (st != HIPMR_OK) return st;

    long long n64 = n, head64 = 0;
    int grid = 0;
    std::string syms;
    if (n > 0) {
        long long head = -1;
        bool vector = h->prog.info.vectorizable && !cfg.force_scalar;
        if (vector) head = common_head(h, args, cfg.vec);
        if (head < 0) vector = false;
        head64 = vector ? head : 0;
        void* fn = nullptr;
        st = variant_function(h, s1_spec(h, vector, cfg, n >= (int64_t(1) << 31), combine, neutral), &fn,
                              &syms);
        if (st != HIPMR_OK) return st;
        long long units = vector ? (n64 > head64 ? (n64 - head64) / cfg.vec : 0) : n64;
        grid = grid_for(units, cfg.block * (vector ? cfg.ipt : 1), cfg, kMaxPartials);
        std::vector<void*> params;
        if (h->prog.sig.args.empty()) params.push_back(&head64);   // hipmr_unused
        for (size_t k = 0; k < h->prog.sig.args.size(); ++k) params.push_back(args[k]);
        params.push_back(&n64);
        params.push_back(&head64);
        params.push_back(&workspace);
        st = launch(fn, (unsigned)grid, (unsigned)cfg.block, params.data(), stream);
        if (st != HIPMR_OK) return st;
    }
    void* fn2 = nullptr;
    st = variant_function(h, s2_spec(combine, neutral), &fn2, &syms);
    if (st != HIPMR_OK) return st;
    set_last_symbols(h, syms);
    void* params2[3] = {&workspace, &grid, &out};
    return launch(fn2, 1, kStage2Block, params2, stream);
}

hipmr_status hipmr_reduce(hipmr_handle h, const char* map_expr, const char* combine,
                          const char* neutral, int64_t n, void* const* args, void* out,
                          void* workspace, size_t workspace_bytes, void* stream) {
    return hipmr_reduce_ex(h, map_expr, combine, neutral, n, args, out, workspace,
                           workspace_bytes, nullptr, stream);
}

const char* hipmr_last_error(void) { return last_error(); }

void hipmr_release(hipmr_handle h) {
    if (h) release_handle(h);
}

hipmr_status hipmr_get_handle_info(hipmr_handle h, hipmr_handle_info* info) {
    clear_error();
    if (!h || !info) return fail(HIPMR_E_INVALID, "NULL argument");
    info->is_reduce = h->prog.sig.is_reduce;
    info->result_dtype = h->prog.sig.result;
    info->nargs = (int32_t)h->prog.sig.args.size();
    info->vectorizable = h->prog.info.vectorizable;
    info->vec = h->default_vec;
    std::string key = h->prog.expr + "\x1f" + std::to_string(h->prog.sig.args.size());
    std::string hex = sha256_hex(key.data(), key.size());
    info->hash = (uint32_t)std::stoul(hex.substr(0, 8), nullptr, 16);
    return HIPMR_OK;
}

hipmr_status hipmr_get_arg_info(hipmr_handle h, int32_t k, int32_t* dtype, int32_t* is_pointer,
                                int32_t* is_const, int32_t* is_read, int32_t* is_written) {
    clear_error();
    if (!h) return fail(HIPMR_E_INVALID, "NULL handle");
    if (k < 0 || k >= (int32_t)h->prog.sig.args.size()) return fail(HIPMR_E_INVALID, "argument index out of range");
    const ArgDecl& a = h->prog.sig.args[k];
    if (dtype) *dtype = a.dtype;
    if (is_pointer) *is_pointer = a.pointer;
    if (is_const) *is_const = a.is_const;
    if (is_read) *is_read = a.read;
    if (is_written) *is_written = a.written;
    return HIPMR_OK;
}

hipmr_status hipmr_get_arg_access(hipmr_handle h, int32_t k, int32_t* access) {
    clear_error();
    if (!h || !access) return fail(HIPMR_E_INVALID, "NULL argument");
    if (k < 0 || k >= (int32_t)h->prog.sig.args.size()) return fail(HIPMR_E_INVALID, "argument index out of range");
    const ArgDecl& a = h->prog.sig.args[k];
    *access = (a.lane ? HIPMR_ACCESS_INDEX : 0) |
              (a.shifted ? HIPMR_ACCESS_SHIFTED : 0) | (a.uniform ? HIPMR_ACCESS_FIXED : 0) |
              (a.other ? HIPMR_ACCESS_OTHER : 0);
    return HIPMR_OK;
}

hipmr_status hipmr_get_kernel_source(hipmr_handle h, int32_t kind, const char* combine,
                                     const char* neutral, char* buf, size_t cap, size_t* len) {
    clear_error();
    if (!h) return fail(HIPMR_E_INVALID, "NULL handle");
    if (kind < 0 || kind > 4) return fail(HIPMR_E_INVALID, "kind must be in 0..4");
    bool red = kind >= 2;
    if (red != (bool)h->prog.sig.is_reduce) return fail(HIPMR_E_MISMATCH, "kind does not match the handle");
    if (red && (!combine || !neutral)) return fail(HIPMR_E_INVALID, "combine_op and neutral are required");
    LaunchCfg cfg;
    resolve_cfg(nullptr, red ? kRedBlock : kEwBlock, red ? kRedIpt : kEwIpt, h->default_vec,
                red ? kRedBlocksPerCu : kEwBlocksPerCu, &cfg);
    KernelSpec spec;
    if (kind == 4) {
        spec = s2_spec(combine, neutral);
    } else if (red) {
        spec = s1_spec(h, kind == 2, cfg, false, combine, neutral);
    } else {
        spec.kind = (KernelKind)kind;
        spec.block = cfg.block;
        spec.ipt = cfg.ipt;
        spec.vec = kind == 0 ? cfg.vec : 1;
    }
    std::string sym;
    std::string src = render(h->prog, spec, &sym);
    if (len) *len = src.size();
    if (buf && cap) {
        size_t c = std::min(cap - 1, src.size());
        std::memcpy(buf, src.data(), c);
        buf[c] = '\0';
    }
    return HIPMR_OK;
}

hipmr_status hipmr_get_last_symbols(hipmr_handle h, char* buf, size_t cap, size_t* len) {
    clear_error();
    if (!h) return fail(HIPMR_E_INVALID, "NULL handle");
    std::string syms;
    {
        std::lock_guard<std::mutex> lk(h->mu);
        syms = h->last_symbols;
    }
    if (len) *len = syms.size();
    if (buf && cap) {
        size_t c = std::min(cap - 1, syms.size());
        std::memcpy(buf, syms.data(), c);
        buf[c] = '\0';
    }
    return HIPMR_OK;
}

hipmr_status hipmr_get_cache_stats(hipmr_cache_stats* out) {
    clear_error();
    if (!out) return fail(HIPMR_E_INVALID, "NULL argument");
    cache_stats(out);
    return HIPMR_OK;
}

void hipmr_cache_drop_memory(void) {
    drop_handle_cache();
    cache_drop_memory();
}

hipmr_status hipmr_sha256_hex(const void* data, size_t len, char* out) {
    clear_error();
    if ((!data && len) || !out) return fail(HIPMR_E_INVALID, "NULL argument");
    std::string h = sha256_hex(data, len);
    std::memcpy(out, h.c_str(), 65);
    return HIPMR_OK;
}

int32_t hipmr_dtype_size(int32_t dtype) { return dtype_size((DType)dtype); }

hipmr_status hipmr_selftest_compile(int32_t* count) {
    clear_error();
    struct Case { const char* expr; const char* dtypes; const char* combine; const char* neutral; };
    static const Case cases[] = {
        {"z[i] = 2.5f*x[i] - 0.5f*y[i]", "float *z, const float *x, const float *y", nullptr, nullptr},
        {"z[i] = sqrtf(x[i]*x[i] + y[i]*y[i])", "float *z, const float *x, const float *y", nullptr, nullptr},
        {"if (k[i] > 3) o[i] = x[i]; else o[i] += 1", "const int *k, const bfloat16 *x, half *o", nullptr, nullptr},
        {"q[i] = x[i + 1 < n ? i + 1 : i] * s", "fp8_e4m3 *q, const float *x, float s", nullptr, nullptr},
        {"int c = i % nx; q[i] = 4.0f*p[i] - (c != 0 ? p[i-1] : 0.0f) - (i + nx < n ? p[i + nx] : 0.0f)",
         "float *q, const float *p, int nx", nullptr, nullptr},
        {"o[i] = 0.5f * (x[i + 2*k] + x[i - (k)])", "bfloat16 *o, const bfloat16 *x, long k", nullptr, nullptr},
        {"k[i] % 7 == 3", "long: const int *k", "a+b", "0"},
        {"x[i]*y[i]", "float: const float *x, const float *y", "a+b", "0"},
        {"x[i]", "float: const float *x", "max(a,b)", "-INFINITY"},
        {"x[i]", "double: const fp8_e4m3 *x", "min", "INFINITY"},
        {"k[i]", "unsigned: const unsigned *k", "a|b", "0u"},
        {"x[n - 1 - i]", "float: const float *x", "a+b", "0"},
        {"(i + 1 < n ? x[i + 1] : 0.0f) * x[i]", "float: const float *x", "a+b", "0"},
        {"x[i]", "float: const fp8_e4m3 *x", "a+b", "0"},
        {"x[i]", "float: const bfloat16 *x", "a+b", "0"},
        {"x[i] * y[i]", "float: const half *x, const half *y", "a+b", "0"},
        {"z[i] = conj(x[i]) * y[i] + a * x[i]", "complex64 *z, const complex64 *x, const complex64 *y, complex64 a",
         nullptr, nullptr},
        {"conj(x[i]) * y[i]", "complex64: const complex64 *x, const complex64 *y", "a+b", "0"},
    };
    int32_t built = 0;
    for (const Case& c : cases) {
        hipmr_handle h = nullptr;
        hipmr_status st = make_handle(c.expr, c.dtypes, "selftest", &h);
        if (st != HIPMR_OK) return st;
        std::shared_ptr<CodeObject> co;
        if (h->prog.sig.is_reduce) {
            LaunchCfg cfg;
            resolve_cfg(nullptr, kRedBlock, kRedIpt, h->default_vec, kRedBlocksPerCu, &cfg);
            for (bool vector : {true, false}) {
                if (vector && !h->prog.info.vectorizable) continue;
                for (bool idx64 : {false, true}) {
                    st = get_variant(h, s1_spec(h, vector, cfg, idx64, c.combine, c.neutral), &co);
                    if (st != HIPMR_OK) { hipmr_release(h); return st; }
                    ++built;
                }
            }
            st = get_variant(h, s2_spec(c.combine, c.neutral), &co);
            ++built;
            if (st == HIPMR_OK) {
                // batching extension: planner, tile stage, per-segment stage
                for (int lds : {0, 4096}) {
                    for (KernelKind k : {KernelKind::SegPlan, KernelKind::SegS1, KernelKind::SegS2}) {
                        KernelSpec q;
                        q.kind = k;
                        q.block = k == KernelKind::SegPlan ? 1024 : 256;
                        q.ipt = k == KernelKind::SegS2 ? 1 : 4;
                        q.vec = k == KernelKind::SegS2 ? 1 : h->default_vec;
                        q.lds_segs = k == KernelKind::SegS1 ? lds : 0;
                        if (k != KernelKind::SegPlan) {
                            q.combine = c.combine;
                            q.neutral = c.neutral;
                        }
                        st = get_variant(h, q, &co);
                        if (st != HIPMR_OK) break;
                        ++built;
                    }
                    if (st != HIPMR_OK) break;
                }
            }
            if (st == HIPMR_OK) {
                // prefix scan: wave totals, their scan, the rescan (vector and scalar)
                for (KernelKind k : {KernelKind::ScanUpVector, KernelKind::ScanUpScalar, KernelKind::ScanMid,
                                     KernelKind::ScanDownVector, KernelKind::ScanDownScalar}) {
                    const bool vk = k == KernelKind::ScanUpVector || k == KernelKind::ScanDownVector;
                    if (vk && !h->prog.info.vectorizable) continue;
                    KernelSpec q;
                    q.kind = k;
                    q.block = k == KernelKind::ScanMid ? 1024 : 256;
                    q.ipt = k == KernelKind::ScanMid ? 1 : 4;
                    q.vec = vk ? h->default_vec : 1;
                    q.combine = c.combine;
                    q.neutral = c.neutral;
                    st = get_variant(h, q, &co);
                    if (st != HIPMR_OK) break;
                    ++built;
                }
            }
            if (st == HIPMR_OK && h->prog.sig.result == DT_F32) {
                // precision extension: compensated sum, norm passes, finishers
                std::vector<KernelSpec> specs;
                for (KernelKind k : {KernelKind::CompS1Vector, KernelKind::CompS1Scalar}) {
                    for (int variant = 0; variant < 3; ++variant) {
                        KernelSpec q = comp_spec(k, cfg);
                        if (k == KernelKind::CompS1Scalar) q.vec = 1;
                        q.square = variant > 0;
                        q.scaled = variant == 2;
                        q.exact_runs = variant == 0 && k == KernelKind::CompS1Vector &&
                                       single_fp8_load(h);
                        specs.push_back(q);
                    }
                }
                for (int variant = 0; variant < 3; ++variant) {
                    KernelSpec q = comp_spec(KernelKind::CompS2, cfg);
                    q.block = kStage2Block;
                    q.ipt = q.vec = 1;
                    q.norm = variant > 0;
                    q.scaled = variant == 2;
                    specs.push_back(q);
                }
                specs.push_back(comp_spec(KernelKind::AmaxS1Vector, cfg));
                for (const KernelSpec& q : specs) {
                    if (!h->prog.info.vectorizable &&
                        (q.kind == KernelKind::CompS1Vector || q.kind == KernelKind::AmaxS1Vector))
                        continue;
                    st = get_variant(h, q, &co);
                    if (st != HIPMR_OK) break;
                    ++built;
                }
            }
        } else {
            KernelSpec spec;
            spec.kind = KernelKind::EwScalar;
            spec.block = kEwBlock;
            spec.ipt = kEwIpt;
            spec.vec = 1;
            st = get_variant(h, spec, &co);
            built += 2;   // + the vector/scalar default built by make_handle
        }
        hipmr_release(h);
        if (st != HIPMR_OK) return st;
    }
    {   // the serving loop's kernels
        hipmr_status st2;
        auto co = get_or_build(serve_source("hipmr_serve"), "hipmr_serve_s1", &st2);
        if (!co) return st2;
        ++built;
    }
    if (count) *count = built;
    return HIPMR_OK;
}

}  // extern "C"
