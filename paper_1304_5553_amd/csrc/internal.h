// Internals shared by the translation units that implement the C ABI:
// the handle object, launch-geometry defaults and the variant cache.
#pragma once

#include <atomic>
#include <map>

#include "common.h"

struct hipmr_kernel {
    int refs = 1;                 // changed only under the handle cache's lock
    bool cached = false;          // listed in the handle cache under cache_key
    std::string cache_key;
    hipmr::Program prog;
    int default_vec = 4;
    std::mutex mu;
    std::map<std::string, std::shared_ptr<hipmr::CodeObject>> variants;
    std::string last_symbols;                        // kernels of the most recent call
    std::map<std::string, hipmr_launch_config> tuned;  // autotuned geometry per operation
};

namespace hipmr {

constexpr int kMaxPartials = 8192;           // stage-1 blocks of one reduce
constexpr int kStage2Block = 256;
// reduce workspace layout: [0, 64 KiB) block partials (FP64 or the
// reduction's type); [64 KiB, 96 KiB) the norm's first-pass partials (max
// |map| per block, float), kept apart so the second pass can read them while
// it writes its own; then the norm's scale as a float (+0) and a double (+8)
constexpr size_t kAmaxOffset = (size_t)kMaxPartials * 8;
constexpr size_t kScaleOffset = kAmaxOffset + (size_t)kMaxPartials * 4;
constexpr size_t kWorkspaceBytes = kScaleOffset + 256;

// Default geometry (overridable per call through hipmr_launch_config), from
// sweeps on MI355X at n = 2^28: streaming reads reach their best rate with a
// small resident grid (2 blocks of 256 threads per CU, 4 chunks of 16 bytes
// in flight per thread and array); elementwise kernels, which mix reads and
// writes, do best as one pass over a full grid (one chunk per thread).
constexpr int kEwBlock = 256, kEwIpt = 1, kEwBlocksPerCu = 1 << 20;
constexpr int kEwScalarBlocksPerCu = 32;     // one-element elementwise kernels
constexpr int kRedBlock = 256, kRedIpt = 4, kRedBlocksPerCu = 2;

hipmr_status resolve_cfg(const hipmr_launch_config* c, int block, int ipt, int vec,
                         int blocks_per_cu, LaunchCfg* out);
hipmr_status get_variant(hipmr_kernel* h, const KernelSpec& spec, std::shared_ptr<CodeObject>* out);
hipmr_status variant_function(hipmr_kernel* h, const KernelSpec& spec, void** fn,
                              std::string* syms);
void set_last_symbols(hipmr_kernel* h, const std::string& syms);
// element offset at which every accessed array is aligned for VEC-element
// chunk loads, or -1
long long common_head(const hipmr_kernel* h, void* const* args, int vec);
hipmr_status check_args(hipmr_kernel* h, int64_t n, void* const* args);
int grid_for(long long work_units, int per_block, const LaunchCfg& cfg, int cap);
// geometry stored by the autotuner for (op, combine, neutral, size class of n)
bool tuned_config(hipmr_kernel* h, const char* op, const char* combine, const char* neutral,
                  long long n, hipmr_launch_config* out);
// cfgp with HIPMR_CFG_TUNED: the stored geometry when one exists and resolves,
// else cfgp without the flag (copied into *buf); any other cfgp unchanged
const hipmr_launch_config* apply_tuned(hipmr_kernel* h, const char* op, const char* combine,
                                       const char* neutral, long long n,
                                       const hipmr_launch_config* cfgp, hipmr_launch_config* buf);

// the segmented map-reduce on a given workspace (hipmr_reduce_segmented's
// body; the no-allocation entry point passes its static scratch array)
size_t segmented_workspace(const hipmr_kernel* h, int32_t nseg, int64_t total_n);
hipmr_status reduce_segmented_on(hipmr_kernel* h, const char* combine, const char* neutral,
                                 int32_t nseg, const int64_t* d_offsets, int64_t total_n,
                                 void* const* args, void* d_out, void* workspace,
                                 size_t workspace_bytes, const hipmr_launch_config* cfgp,
                                 void* stream);

// device source of the serving loop's kernels
std::string serve_source(const std::string& prefix);

}  // namespace hipmr
