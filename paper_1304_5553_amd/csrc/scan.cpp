// Prefix scan of a map (the parallel prefix sums the paper lists among the
// facilities built from the same ingredients as the map-reduce: a map over
// the formal index i, a combine in a and b, its neutral element; section
// "Further Facilities" with section "Map-Reduce").
//
// Reduce-then-scan in four launches, deterministic and without atomics:
//   1. scu / scus: each wave folds its contiguous range into partial[w];
//   2. scm:        each block of 1024 wave totals is scanned (exclusive), then
//                  one block scans the block totals (a second scm launch);
//   3. scd / scds: each wave rescans its range from its prefix and writes out.
// The partition depends only on n, the alignment head and the geometry, so a
// result is bitwise repeatable.  The input is read twice and the output
// written once.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <vector>

#include "internal.h"

using namespace hipmr;

namespace {

// Many short ranges (up to 65536 waves): the waves running together cover a
// compact address window, which keeps the writes efficient (measured on
// MI355X: a copy with this partition loses ~20 % when each wave owns 64 KB
// instead of 4-16 KB).  Passes of 4 sub-tiles per wave; pass 1 takes at most
// 4 sub-tiles per step whatever the pass-3 geometry.
constexpr int kScanBlock = 256, kScanIpt = 4, kScanUpIpt = 4;
constexpr long long kScanMaxWaves = 65536;   // wave totals (pass 2: 64 blocks of 1024)
constexpr int kScanMidBlock = 1024;

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Element offset at which every accessed array and the output are aligned
// for VEC-element chunks, or -1.
long long scan_head(const hipmr_kernel* h, void* const* args, const void* out, int vec) {
    const int rs = dtype_size(h->prog.sig.result);
    for (long long head = 0; head < vec; ++head) {
        bool ok = true;
        for (size_t k = 0; k < h->prog.sig.args.size() && ok; ++k) {
            const ArgDecl& a = h->prog.sig.args[k];
            if (!chunked(a)) continue;
            uintptr_t p = (uintptr_t)(*(void* const*)args[k]);
            int s = dtype_size(a.dtype);
            uintptr_t align = (uintptr_t)std::min(vec * s, 16);
            if (p % (uintptr_t)s != 0 || (p + (uintptr_t)head * s) % align != 0) ok = false;
        }
        uintptr_t o = (uintptr_t)out;
        if (o % (uintptr_t)rs != 0 || (o + (uintptr_t)head * rs) % 16 != 0) ok = false;
        if (ok) return head;
    }
    return -1;
}

KernelSpec scan_spec(KernelKind kind, const LaunchCfg& cfg, bool idx64, const char* combine,
                     const char* neutral) {
    KernelSpec s;
    s.kind = kind;
    s.idx64 = idx64;
    s.block = kind == KernelKind::ScanMid ? kScanMidBlock : cfg.block;
    s.ipt = kind == KernelKind::ScanMid ? 1 : cfg.ipt;
    s.vec = kind == KernelKind::ScanMid ? 1 : cfg.vec;
    s.nt_loads = kind == KernelKind::ScanMid ? true : cfg.nt_loads;
    s.nt_stores = kind == KernelKind::ScanMid ? true : cfg.nt_stores;
    s.combine = combine;
    s.neutral = neutral;
    return s;
}

}  // namespace

extern "C" {

size_t hipmr_scan_workspace_bytes(hipmr_handle h, int64_t n) {
    if (!h || !h->prog.sig.is_reduce || n < 0) return 0;
    const size_t rs = (size_t)dtype_size(h->prog.sig.result);
    // wave totals, wave prefixes within their block of 1024, block prefixes
    return 2 * align256((size_t)kScanMaxWaves * rs) + align256((size_t)(kScanMaxWaves / 1024) * rs);
}

hipmr_status hipmr_scan(hipmr_handle h, const char* combine, const char* neutral, int64_t n,
                        void* const* args, void* out, int32_t exclusive, void* workspace,
                        size_t workspace_bytes, const hipmr_launch_config* cfgp, void* stream) {
    clear_error();
    hipmr_status st = check_args(h, n, args);
    if (st != HIPMR_OK) return st;
    if (!h->prog.sig.is_reduce) return fail(HIPMR_E_MISMATCH, "elementwise handle passed to hipmr_scan");
    if (!combine || !neutral) return fail(HIPMR_E_INVALID, "combine_op and neutral are required");
    if (exclusive != 0 && exclusive != 1) return fail(HIPMR_E_INVALID, "exclusive must be 0 or 1");
    if (n == 0) return HIPMR_OK;
    if (!out) return fail(HIPMR_E_INVALID, "out is NULL");
    if (!workspace || workspace_bytes < hipmr_scan_workspace_bytes(h, n))
        return fail(HIPMR_E_WORKSPACE, "workspace smaller than hipmr_scan_workspace_bytes()");
    // Default chunk: 16 bytes of the narrowest input, but at most 16 bytes of
    // output per lane, so that each store instruction of a wave writes one
    // contiguous run; a narrower chunk takes more sub-tiles per pass (at most
    // 8) to keep the loads in flight.
    const int out_size = dtype_size(h->prog.sig.result);
    const int dvec = std::min(h->default_vec, std::max(1, 16 / out_size));
    const int dipt = std::min(8, kScanIpt * (h->default_vec / dvec));
    LaunchCfg cfg;
    st = resolve_cfg(cfgp, kScanBlock, dipt, dvec, 1, &cfg);
    if (st != HIPMR_OK) return st;

    long long head = h->prog.info.vectorizable && !cfg.force_scalar ? scan_head(h, args, out, cfg.vec) : -1;
    const bool vector = head >= 0;
    if (!vector) {
        cfg.vec = 1;
        head = 0;
    }
    const long long n64 = n;
    head = std::min<long long>(head, n64);
    const long long body = n64 - head;
    const long long sub = 64LL * cfg.vec * cfg.ipt;            // one pass of a wave (pass 3)
    const long long passes = std::max<long long>(1, (body + sub * kScanMaxWaves - 1) / (sub * kScanMaxWaves));
    const long long waves = std::max<long long>(1, (body + sub * passes - 1) / (sub * passes));
    int passes32 = (int)passes;
    // pass 1 covers the same ranges in steps of at most kScanUpIpt sub-tiles
    LaunchCfg up = cfg;
    up.ipt = std::min(cfg.ipt, kScanUpIpt);
    while (cfg.ipt % up.ipt) --up.ipt;
    int passes_up = (int)(passes * (cfg.ipt / up.ipt));
    const bool idx64 = n64 >= (int64_t(1) << 31);

    std::string syms;
    void *f_up = nullptr, *f_mid = nullptr, *f_down = nullptr;
    st = variant_function(h, scan_spec(vector ? KernelKind::ScanUpVector : KernelKind::ScanUpScalar, up,
                                       idx64, combine, neutral), &f_up, &syms);
    if (st != HIPMR_OK) return st;
    st = variant_function(h, scan_spec(KernelKind::ScanMid, cfg, false, combine, neutral), &f_mid, &syms);
    if (st != HIPMR_OK) return st;
    st = variant_function(h, scan_spec(vector ? KernelKind::ScanDownVector : KernelKind::ScanDownScalar, cfg,
                                       idx64, combine, neutral), &f_down, &syms);
    if (st != HIPMR_OK) return st;
    set_last_symbols(h, syms);

    const size_t rs = (size_t)dtype_size(h->prog.sig.result);
    void* partial = workspace;
    void* prefix = (char*)workspace + align256((size_t)kScanMaxWaves * rs);
    void* bpre = (char*)prefix + align256((size_t)kScanMaxWaves * rs);
    const unsigned grid = (unsigned)((waves + cfg.block / 64 - 1) / (cfg.block / 64));
    long long waves64 = waves;
    int excl = exclusive;

    std::vector<void*> p1;
    if (h->prog.sig.args.empty()) p1.push_back(&head);       // hipmr_unused
    for (size_t k = 0; k < h->prog.sig.args.size(); ++k) p1.push_back(args[k]);
    std::vector<void*> p3 = p1;
    long long n_arg = n64;
    p1.insert(p1.end(), {(void*)&n_arg, (void*)&head, (void*)&passes_up, (void*)&waves64, (void*)&partial});
    st = launch(f_up, grid, (unsigned)cfg.block, p1.data(), stream);
    if (st != HIPMR_OK) return st;
    int top0 = 0, top1 = 1;
    void* p2a[5] = {&partial, &waves64, &prefix, &bpre, &top0};
    st = launch(f_mid, (unsigned)((waves + 1023) / 1024), kScanMidBlock, p2a, stream);
    if (st != HIPMR_OK) return st;
    void* p2b[5] = {&partial, &waves64, &prefix, &bpre, &top1};
    st = launch(f_mid, 1, kScanMidBlock, p2b, stream);
    if (st != HIPMR_OK) return st;
    p3.insert(p3.end(), {(void*)&n_arg, (void*)&head, (void*)&passes32, (void*)&waves64, (void*)&prefix,
                         (void*)&bpre, (void*)&out, (void*)&excl});
    return launch(f_down, grid, (unsigned)cfg.block, p3.data(), stream);
}

}  // extern "C"
