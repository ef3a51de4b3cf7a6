// Serving extension: a request loop for map-reduce jobs with continuous
// batching.
//
// Jobs are map-reduce requests of one of eight templates over flat float32 or
// bfloat16 arrays that stay resident on the device:
//   sum, dot, L2 norm, max, axpby-then-sum, count(x > 0), sum of squares and
//   weighted mean.
// A host thread owns the loop:
//   - arrivals are released at their scheduled time;
//   - they are admitted while the bytes of unfinished jobs stay within the HBM
//     budget;
//   - admitted jobs go to the free stream slots, one batch per slot (up to k
//     batches in flight): one job per slot while the queue is short, batches
//     of ceil(waiting / free slots) once it is long, so batches grow with the
//     backlog; a large job runs in a batch of its own and small jobs are
//     packed past it;
//   - a batch is two launches of run-time compiled kernels:
//       1. a persistent kernel whose waves take fixed-size tiles of any job in
//          the batch (a wave-uniform switch over template x dtype);
//       2. one block per job folding that job's tile partials in a fixed
//          order and finishing the job (sqrt, ratio);
//   - completion is observed through per-job flags in mapped host memory,
//     written by the finishing block after the result (querying the stream
//     serves as a watchdog for errors).
// A job's tiles depend only on the job (its length, dtype and alignment; big
// jobs get longer tiles so that none has more than 4080), so its result is
// bitwise the same alone or in any mix.  A batch of one job passes its
// descriptor by value; with max_batch_jobs = 1 every job runs that way, one
// launch pair per job: the baseline.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <vector>
#include <thread>

#include "internal.h"

using namespace hipmr;

namespace {

constexpr int kServeBlock = 256;          // tile kernels: 4 waves, one tile per wave at a time
constexpr int kFinBlock = 1024;           // final fold: one block per job
constexpr int kMaxBatchJobs = 4096;      // jobs per batch (their tile offsets are staged in LDS)
constexpr int kInlineJobs = 24;          // descriptors passed as kernel arguments
constexpr int kMaxSkipped = 64;          // large jobs one batch of small ones may be packed past
constexpr int kOneLaunchTiles = 16;      // a job of at most this many tiles alone: one launch
constexpr int64_t kWatchdogNs = 20000000;  // after 20 ms without flags, query the stream
constexpr int kRoundTiles = 4080;        // tiles of one job at most: a round of the resident kernel
                                         // (255 worker CUs x 16 waves, one tile each)
constexpr long long kMaxBaseTiles = 65536;  // one-pass tiles of the largest job (2^26 f32, 2^27 bf16)
constexpr int kRing = 4096;               // resident: job descriptors in flight (power of two)
constexpr int kRingWords = 16;            // resident: 64-bit words per host ring slot (nine used)
constexpr uint64_t kField = (1ull << 48) - 1;   // resident: a ring word's payload
constexpr size_t kCtrlBytes = 4096;       // resident: control words (zeroed before each launch)
constexpr int64_t kRotateNs = 250000000;  // resident: a new instance every 250 ms of service
constexpr int64_t kIdleStopNs = 10000000; // resident: the instance stops after 10 ms without jobs
constexpr double kLifeS = 2.0;            // resident: an instance's deadline (it exits by then)
constexpr int kEpochShift = 44;           // resident: stop / exit words = epoch << 44 | job index

// Device descriptor of one job (64 bytes; the layout matches the device-side
// hipmr_sjob struct in the kernels below).
struct DevJob {
    const void* x;
    const void* y;
    const void* w;
    long long n;
    int tmpl;
    int dtype;
    int tile0;
    int head;
    double* out;
    float a, b;
};
static_assert(sizeof(DevJob) == 64, "job descriptor layout");

struct InlineJobs {
    int njobs, total_tiles, pad0, pad1;
    DevJob jobs[kInlineJobs];
};

const char* kServeKernels = R"HIP(
struct hipmr_sjob {
  const void* x; const void* y; const void* w;
  long long n;
  int tmpl, dtype, tile0, head;
  double* out;
  float a, b;
};

// Lane moves (every lane of the wave active): DPP inside rows of 16 lanes,
// v_readlane for one lane's value.
template <int CTRL>
__device__ __forceinline__ unsigned hipmr_dpp32(unsigned v) {
  return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ float hipmr_dpp(float v) {
  return __builtin_bit_cast(float, hipmr_dpp32<CTRL>(__builtin_bit_cast(unsigned, v)));
}
template <int CTRL>
__device__ __forceinline__ double hipmr_dpp(double v) {
  const unsigned long long a = __builtin_bit_cast(unsigned long long, v);
  return __builtin_bit_cast(double, (unsigned long long)hipmr_dpp32<CTRL>((unsigned)(a >> 32)) << 32 |
                                        hipmr_dpp32<CTRL>((unsigned)a));
}
__device__ __forceinline__ unsigned long long hipmr_readlane64(unsigned long long v, int l) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), l);
  return (unsigned long long)hi << 32 | lo;
}
__device__ __forceinline__ float hipmr_rl(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double hipmr_rl(double v, int l) {
  return __builtin_bit_cast(double, hipmr_readlane64(__builtin_bit_cast(unsigned long long, v), l));
}

// Butterfly fold of a commutative op over the wave, lane distance 1, 2, 4, 8
// (DPP quad permutations, then the half-row and row mirrors: once each quad,
// then each half-row, holds one value, the mirror partner is as good as the
// xor partner), then 16 and 32 (one lane read from each row).  Every lane
// ends with the same value; the tree has depth 6.
template <typename T, typename Op>
__device__ __forceinline__ T hipmr_wave_fold(T v, Op op) {
  v = op(v, hipmr_dpp<0xb1>(v));         // lane ^ 1
  v = op(v, hipmr_dpp<0x4e>(v));         // lane ^ 2
  v = op(v, hipmr_dpp<0x141>(v));        // the other quad of the half-row
  v = op(v, hipmr_dpp<0x140>(v));        // the other half of the row
  return op(op(hipmr_rl(v, 0), hipmr_rl(v, 16)), op(hipmr_rl(v, 32), hipmr_rl(v, 48)));
}

// One element's terms (t0, t1) under template TMPL; t1 is the weight of the
// weighted mean and 0 otherwise.
template <int TMPL>
__device__ __forceinline__ float2 hipmr_job_term(float x, float y, float w, float a, float b) {
  if constexpr (TMPL == 0 || TMPL == 3) return make_float2(x, 0.0f);  // sum, max
  else if constexpr (TMPL == 1) return make_float2(x * y, 0.0f);      // dot
  else if constexpr (TMPL == 2 || TMPL == 6) return make_float2(x * x, 0.0f);  // norm, sum of squares
  else if constexpr (TMPL == 4) return make_float2(a * x + b * y, 0.0f);       // axpby, then sum
  else if constexpr (TMPL == 5) return make_float2(x > 0.0f ? 1.0f : 0.0f, 0.0f);  // count(x > 0)
  else return make_float2(w * x, w);                                  // weighted mean
}

template <int TMPL>
__device__ __forceinline__ float hipmr_job_comb(float a, float b) {
  if constexpr (TMPL == 3) return __builtin_elementwise_maximum(a, b);
  else return a + b;
}

template <int TMPL>
__device__ __forceinline__ float2 hipmr_job_comb2(float2 a, float2 b) {
  return make_float2(hipmr_job_comb<TMPL>(a.x, b.x), a.y + b.y);
}

// Tile geometry of a job, a function of the job alone: `ab` unaligned head
// elements (all arrays 16-byte aligned after them; 0 when they share no
// alignment), then tiles of `tt` elements = Q chunks of V elements per lane
// x 64 lanes, taken in P = ceil(Q / 4) passes of up to 4 chunks per lane.
// Q is 4 while that keeps the job at or under 4080 tiles (up to 2^22 float32
// / 2^23 bfloat16 elements), else the smallest that does (17 at 2^24 float32
// elements, 65 at 2^26, the largest job taken): the resident kernel's 4080
// waves take every job in one round.  Arrays without a common alignment take
// their tiles element by element.
struct hipmr_geom { long long ab, tt; int passes, tiles; };

__device__ __forceinline__ hipmr_geom hipmr_job_geom(const hipmr_sjob& J) {
  const int lg = J.dtype == @@BF16CODE@@ ? 9 : 8;        // one chunk per lane: 2^lg elements
  hipmr_geom g;
  g.ab = J.head >= 0 ? (J.head < J.n ? J.head : J.n) : 0;
  const long long body = J.n - g.ab;
  const long long c1 = (body + (1ll << lg) - 1) >> lg;
  const int q = c1 > 4 * @@ROUND_TILES@@ ? (int)((c1 + @@ROUND_TILES@@ - 1) / @@ROUND_TILES@@) : 4;
  g.passes = (q + 3) / 4;
  g.tt = (long long)q << lg;
  // ceil(body / (q 2^lg)) = ceil(c1 / q); c1 <= 2^18 for every job admitted
  const long long t = q == 4 ? (c1 + 3) >> 2 : (long long)(((unsigned)c1 + (unsigned)q - 1) / (unsigned)q);
  g.tiles = J.n <= 0 ? 0 : (t < 1 ? 1 : (int)t);
  return g;
}

// Tile k of job J, reduced by one wave.  Tile 0 also holds the unaligned
// head.  Lane l takes chunks l + 64 (u + 4 p) of the tile; each chunk's V
// terms are summed pairwise, then added to accumulator u (one per chunk
// slot, across the P passes); the 4 accumulators fold pairwise, then across
// the wave.  Every float sum on the way has depth <= P + 11 (28 at most).
// The last pass may hold fewer than 4 chunks per lane.
template <int TMPL, typename T, int V>
__device__ __forceinline__ float2 hipmr_job_tile(const hipmr_sjob& J, long long k, int lane) {
  constexpr int U = 4;
  constexpr bool NY = TMPL == 1 || TMPL == 4, NW = TMPL == 7;
  const T* X = (const T*)J.x;
  const T* Y = (const T*)J.y;
  const T* W = (const T*)J.w;
  const hipmr_geom g = hipmr_job_geom(J);
  const long long n = J.n;
  const long long ts = k == 0 ? 0 : g.ab + k * g.tt;
  const long long te = g.ab + (k + 1) * g.tt < n ? g.ab + (k + 1) * g.tt : n;
  const float neutral = TMPL == 3 ? -__builtin_huge_valf() : 0.0f;
  float2 acc[U];
#pragma unroll
  for (int u = 0; u < U; ++u) acc[u] = make_float2(neutral, 0.0f);
  auto elem = [&](long long e) {
    return hipmr_job_term<TMPL>((float)X[e], NY ? (float)Y[e] : 0.0f, NW ? (float)W[e] : 0.0f, J.a, J.b);
  };
  if (J.head < 0) {                      // arrays without a common alignment: single elements
    for (long long e0 = ts + lane; e0 < te; e0 += 64 * U) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (e0 + 64 * u < te) acc[u] = hipmr_job_comb2<TMPL>(acc[u], elem(e0 + 64 * u));
    }
  } else {
    const long long hend = k == 0 ? g.ab : ts;
    const long long nch = te > hend ? (te - hend) / V : 0;
    const long long tail = hend + nch * V;
    if (lane < hend - ts) acc[0] = hipmr_job_comb2<TMPL>(acc[0], elem(ts + lane));
    for (int p = 0; p < g.passes; ++p) {
      hipmr_pack<T, V> px[U], py[U], pw[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const long long c = lane + 64 * (u + U * p);
        if (c < nch) {
          const long long off = hend + c * V;
          hipmr_load<true>(px[u], X + off);
          if constexpr (NY) hipmr_load<true>(py[u], Y + off);
          if constexpr (NW) hipmr_load<true>(pw[u], W + off);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const long long c = lane + 64 * (u + U * p);
        if (c < nch) {
          float2 t[V];
#pragma unroll
          for (int j = 0; j < V; ++j)
            t[j] = hipmr_job_term<TMPL>((float)px[u].v[j], NY ? (float)py[u].v[j] : 0.0f,
                                        NW ? (float)pw[u].v[j] : 0.0f, J.a, J.b);
#pragma unroll
          for (int w = 1; w < V; w *= 2) {
#pragma unroll
            for (int j = 0; j + w < V; j += 2 * w) t[j] = hipmr_job_comb2<TMPL>(t[j], t[j + w]);
          }
          acc[u] = hipmr_job_comb2<TMPL>(acc[u], t[0]);
        }
      }
    }
    if (lane < te - tail) acc[U - 1] = hipmr_job_comb2<TMPL>(acc[U - 1], elem(tail + lane));
  }
  acc[0] = hipmr_job_comb2<TMPL>(acc[0], acc[1]);
  acc[2] = hipmr_job_comb2<TMPL>(acc[2], acc[3]);
  float2 r = hipmr_job_comb2<TMPL>(acc[0], acc[2]);
  r.x = hipmr_wave_fold(r.x, [](float p, float q) { return hipmr_job_comb<TMPL>(p, q); });
  r.y = hipmr_wave_fold(r.y, [](float p, float q) { return p + q; });
  return r;
}

__device__ __forceinline__ float2 hipmr_job_dispatch(const hipmr_sjob& J, long long k, int lane) {
  const bool bf = J.dtype == @@BF16CODE@@;
  switch (J.tmpl * 2 + (bf ? 1 : 0)) {
    case 0: return hipmr_job_tile<0, float, 4>(J, k, lane);
    case 1: return hipmr_job_tile<0, hipmr_bf16, 8>(J, k, lane);
    case 2: return hipmr_job_tile<1, float, 4>(J, k, lane);
    case 3: return hipmr_job_tile<1, hipmr_bf16, 8>(J, k, lane);
    case 4: return hipmr_job_tile<2, float, 4>(J, k, lane);
    case 5: return hipmr_job_tile<2, hipmr_bf16, 8>(J, k, lane);
    case 6: return hipmr_job_tile<3, float, 4>(J, k, lane);
    case 7: return hipmr_job_tile<3, hipmr_bf16, 8>(J, k, lane);
    case 8: return hipmr_job_tile<4, float, 4>(J, k, lane);
    case 9: return hipmr_job_tile<4, hipmr_bf16, 8>(J, k, lane);
    case 10: return hipmr_job_tile<5, float, 4>(J, k, lane);
    case 11: return hipmr_job_tile<5, hipmr_bf16, 8>(J, k, lane);
    case 12: return hipmr_job_tile<6, float, 4>(J, k, lane);
    case 13: return hipmr_job_tile<6, hipmr_bf16, 8>(J, k, lane);
    case 14: return hipmr_job_tile<7, float, 4>(J, k, lane);
    default: return hipmr_job_tile<7, hipmr_bf16, 8>(J, k, lane);
  }
}

// Final fold of one job's tile partials, the same arithmetic on every path
// (launched batches, one launch per job, the resident kernel), so a job's
// result never depends on the path that ran it.  FP64, in two levels:
//   1. group g of 64 consecutive tiles: lane l holds partial 64 g + l (the
//      neutral element past the job's last tile), then the wave butterfly;
//   2. the groups (at most 64, as a job has at most 4080 tiles; room for
//      128): lane l
//      folds the neutral element, group l and group l + 64 in that order,
//      then the wave butterfly.
// Every lane ends with the same value.  The second component (the weight of
// the weighted mean, 0 otherwise) always sums.
__device__ __forceinline__ double2 hipmr_fin_comb(bool mx, double2 a, double2 b) {
  return make_double2(mx ? __builtin_elementwise_maximum(a.x, b.x) : a.x + b.x, a.y + b.y);
}

__device__ __forceinline__ double2 hipmr_fin_wave(bool mx, double2 v) {
  const auto plus = [](double p, double q) { return p + q; };
  v.x = mx ? hipmr_wave_fold(v.x, [](double p, double q) { return __builtin_elementwise_maximum(p, q); })
           : hipmr_wave_fold(v.x, plus);
  v.y = hipmr_wave_fold(v.y, plus);
  return v;
}

__device__ __forceinline__ double2 hipmr_fin_neutral(bool mx) {
  return make_double2(mx ? -__builtin_huge_val() : 0.0, 0.0);
}

// Level 1: group g of a job whose partial k sits at tpart[(base + k) & mask].
__device__ __forceinline__ double2 hipmr_fin_group(bool mx, const float2* tpart, unsigned long long base,
                                                   unsigned long long mask, int g, int ntiles, int lane) {
  const int k = 64 * g + lane;
  double2 v = hipmr_fin_neutral(mx);
  if (k < ntiles) {
    const float2 p = tpart[(base + (unsigned long long)k) & mask];
    v = make_double2((double)p.x, (double)p.y);
  }
  return hipmr_fin_wave(mx, v);
}

// Level 2: lane l holds group l (if h0) and group l + 64 (if h1).
__device__ __forceinline__ double2 hipmr_fin_level2(bool mx, bool h0, double2 v0, bool h1, double2 v1) {
  double2 a = hipmr_fin_neutral(mx);
  if (h0) a = hipmr_fin_comb(mx, a, v0);
  if (h1) a = hipmr_fin_comb(mx, a, v1);
  return hipmr_fin_wave(mx, a);
}

// Level 2 over the ng group values gv[0 .. ng).
__device__ __forceinline__ double2 hipmr_fin_groups(bool mx, const double2* gv, int ng, int lane) {
  const bool h0 = lane < ng, h1 = lane + 64 < ng;
  const double2 z = make_double2(0.0, 0.0);
  return hipmr_fin_level2(mx, h0, h0 ? gv[lane] : z, h1, h1 ? gv[lane + 64] : z);
}

// The job's result from its total (square root of the norm, ratio of the
// weighted mean), written before the job's completion flag (in host memory)
// changes.  The result goes out as a system-scope store, which completes
// only once it is visible to the whole system, so waiting for it (rather
// than a system-scope fence, which writes back the whole L2) orders it
// before the flag.
__device__ __forceinline__ void hipmr_job_post_to(int tmpl, double* out, double2 tot,
                                                  unsigned long long* flag, unsigned long long seq) {
  double r = tot.x;
  if (tmpl == 2) r = sqrt(r);
  else if (tmpl == 7) r = r / tot.y;
  __hip_atomic_store((unsigned long long*)out, __builtin_bit_cast(unsigned long long, r), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_SYSTEM);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __hip_atomic_store(flag, seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void hipmr_job_post(const hipmr_sjob& J, double2 tot,
                                               unsigned long long* flag, unsigned long long seq) {
  hipmr_job_post_to(J.tmpl, J.out, tot, flag, seq);
}

// The fold of the partials [t0, t1) by one block of 1024 threads: wave w
// takes groups w, w + 16, ... (the loads of up to four issued together);
// wave 0 then folds the groups and finishes.
constexpr int HIPMR_FIN_BLOCK = 1024;

__device__ __forceinline__ void hipmr_job_finish(const hipmr_sjob& J, int t0, int t1,
                                                 const float2* __restrict__ tpart,
                                                 unsigned long long* flag, unsigned long long seq) {
  __shared__ double2 hipmr_gv[128];
  const bool mx = J.tmpl == 3;
  const int ntiles = t1 - t0, ng = (ntiles + 63) / 64;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  constexpr int S = HIPMR_FIN_BLOCK / 64;
  for (int g0 = w; g0 < ng; g0 += 4 * S) {
    // unconditional loads (the index clamped into [t0, t1)), so that no
    // branch separates them and all four are in flight together
    float2 p[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = 64 * (g0 + S * i) + lane;
      p[i] = tpart[t0 + (k < ntiles ? k : ntiles - 1)];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int g = g0 + S * i, k = 64 * g + lane;
      if (g < ng) {                       // the fold of hipmr_fin_group
        const double2 v = hipmr_fin_wave(mx, k < ntiles ? make_double2((double)p[i].x, (double)p[i].y)
                                                        : hipmr_fin_neutral(mx));
        if (lane == 0) hipmr_gv[g] = v;
      }
    }
  }
  __syncthreads();
  if (w == 0) {
    const double2 tot = hipmr_fin_groups(mx, hipmr_gv, ng, lane);
    if (lane == 0) hipmr_job_post(J, tot, flag, seq);
  }
}

// Batched stage 1: persistent waves over the batch's tiles.
extern "C" __global__ void __launch_bounds__(256)
@@PREFIX@@_s1(const hipmr_sjob* __restrict__ jobs, int njobs, int total_tiles,
              float2* __restrict__ tpart)
{
  extern __shared__ int hipmr_t0[];             // njobs entries (dynamic LDS)
  for (int k = threadIdx.x; k < njobs; k += 256) hipmr_t0[k] = jobs[k].tile0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int nwaves = gridDim.x * 4;
  for (int t = blockIdx.x * 4 + (threadIdx.x >> 6); t < total_tiles; t += nwaves) {
    int lo = 0, hi = njobs - 1;                 // the last job with tile0 <= t
    while (lo < hi) {
      const int step = (hi - lo + 64) / 64;
      const int cand = lo + lane * step;
      const bool pred = cand <= hi && hipmr_t0[cand] <= t;
      const unsigned long long m = __ballot(pred);
      lo = lo + (63 - __builtin_clzll(m)) * step;
      hi = lo + step - 1 < hi ? lo + step - 1 : hi;
    }
    const hipmr_sjob J = jobs[lo];
    const float2 r = hipmr_job_dispatch(J, t - J.tile0, lane);
    if (lane == 0) tpart[t] = r;
  }
}

// Batched stage 2: one wave per job.
extern "C" __global__ void __launch_bounds__(1024)
@@PREFIX@@_s2(const hipmr_sjob* __restrict__ jobs, int njobs, int total_tiles,
              const float2* __restrict__ tpart, unsigned long long* flags, unsigned long long seq)
{
  const int j = blockIdx.x;                     // one block per job (grid = njobs)
  const hipmr_sjob J = jobs[j];
  const int t1 = j + 1 < njobs ? jobs[j + 1].tile0 : total_tiles;
  hipmr_job_finish(J, J.tile0, t1, tpart, flags + j, seq);
}

// Small batches: the descriptors travel by value in the kernel arguments
// (no separate host-to-device copy before the launch).
struct hipmr_jobs_inline {
  int njobs, total_tiles, pad0, pad1;
  hipmr_sjob jobs[@@NINLINE@@];
};

extern "C" __global__ void __launch_bounds__(256)
@@PREFIX@@_i1(const hipmr_jobs_inline B, float2* __restrict__ tpart)
{
  const int lane = threadIdx.x & 63;
  const int nwaves = gridDim.x * 4;
  for (int t = blockIdx.x * 4 + (threadIdx.x >> 6); t < B.total_tiles; t += nwaves) {
    int j = 0;                                  // the last job with tile0 <= t
    for (int k = 1; k < B.njobs; ++k) j = B.jobs[k].tile0 <= t ? k : j;
    const hipmr_sjob J = B.jobs[j];
    const float2 r = hipmr_job_dispatch(J, t - J.tile0, lane);
    if (lane == 0) tpart[t] = r;
  }
}

extern "C" __global__ void __launch_bounds__(1024)
@@PREFIX@@_i2(const hipmr_jobs_inline B, const float2* __restrict__ tpart,
              unsigned long long* flags, unsigned long long seq)
{
  const int j = blockIdx.x;                     // one block per job (grid = njobs)
  const hipmr_sjob J = B.jobs[j];
  const int t1 = j + 1 < B.njobs ? B.jobs[j + 1].tile0 : B.total_tiles;
  hipmr_job_finish(J, J.tile0, t1, tpart, flags + j, seq);
}

// A small job in one launch: one block of 1024 threads computes the tile
// partials (tile t by wave t mod 16, the arithmetic of the tile kernels) and,
// after a barrier, folds them as the fold kernels do, so the result is
// bitwise the one of any other path.
extern "C" __global__ void __launch_bounds__(1024)
@@PREFIX@@_one(hipmr_sjob J, float2* __restrict__ tpart, unsigned long long* flags,
               unsigned long long seq)
{
  const int lane = threadIdx.x & 63;
  const int tiles = hipmr_job_geom(J).tiles;
  for (int t = threadIdx.x >> 6; t < tiles; t += HIPMR_FIN_BLOCK / 64) {
    const float2 r = hipmr_job_dispatch(J, t, lane);
    if (lane == 0) tpart[t] = r;
  }
  __syncthreads();
  hipmr_job_finish(J, 0, tiles, tpart, flags, seq);
}

// One job, descriptor by value: the one-launch-pair-per-job path.
extern "C" __global__ void __launch_bounds__(256)
@@PREFIX@@_one1(hipmr_sjob J, float2* __restrict__ tpart)
{
  const int lane = threadIdx.x & 63;
  const int tiles = hipmr_job_geom(J).tiles;
  for (int t = blockIdx.x * 4 + (threadIdx.x >> 6); t < tiles; t += gridDim.x * 4) {
    const float2 r = hipmr_job_dispatch(J, t, lane);
    if (lane == 0) tpart[t] = r;
  }
}

extern "C" __global__ void __launch_bounds__(1024)
@@PREFIX@@_one2(hipmr_sjob J, const float2* __restrict__ tpart, unsigned long long* flags,
                unsigned long long seq)
{
  hipmr_job_finish(J, 0, hipmr_job_geom(J).tiles, tpart, flags, seq);
}

// ---------------------------------------------------------------- resident
// One kernel that stays on the device and takes jobs from a ring of
// descriptors in mapped host memory, so a job costs no launch.
//   Host ring (mapped host memory): job s sits in slot s % R of hr_words as
//   nine 64-bit words (x, y, w, n, out, tmpl | dtype << 8 | head << 16 |
//   epoch << 32 (head a signed 16-bit field, epoch the low 16 bits of the
//   instance the job was written for), a, b, its first tile's global
//   index), each a 48-bit field under a 16-bit
//   tag of its lap of the ring ((s / R + 1) mod 2^16): one read of the nine
//   words finds a job complete when every word carries its lap's tag, so
//   the dispatcher needs no separate published count (and no second trip
//   over PCIe);
//   hdr[16] = epoch << 44 | the job index at which instance `epoch` stops
//   accepting (a word naming another epoch does not stop this one); the
//   dispatcher writes hdr[32] = epoch << 44 | (jobs accepted + 1) as it
//   exits; hr_flags[slot] = s + 1 once job s's result is in device memory.
//   Control words (device memory, zeroed before each launch): ctrl[0] tile
//   tickets taken; ctrl[16] jobs completed; eight replicas (one line each,
//   ctrl[32 + 16 r]) of {published: jobs (relative to job_base) << 40 | tiles
//   (relative to tile_base), in one word so the two always agree; stop}.
// Block 0, wave 0 is the dispatcher: it copies newly published descriptors
// into the device ring and publishes them; once the host's stop index is
// reached and every accepted job has completed (or at its deadline), it sets
// the stop flag and exits.  Blocks 1.. are workers: thread 0 takes 16
// consecutive tile tickets (one per wave) and polls the block's replica until
// they are published; each wave reduces its tile with the tile kernels'
// arithmetic; then wave 0 counts the round's tiles into their 64-tile groups
// (one atomic per group touched), folds each group the round completed, and
// the wave completing a job's last group folds the groups and writes the
// result (the fold of every other path).  Every wait is bounded: workers exit
// on the stop flag, and every wave at the instance's deadline.
//
// Memory ordering without cache maintenance: everything one wave hands to
// another (descriptors, first tiles, tile partials, group values, counters,
// the published word) is written and read with device-scope atomic accesses,
// which the L2 keeps coherent across the chip's dies; a writer waits for its
// data writes to complete (s_waitcnt) before the atomic that publishes them,
// and a reader issues its data reads only after that atomic's value is
// known.  (Acquire / release fences at device scope would write back and
// invalidate the whole L2 at every tile.)
#define HIPMR_RING @@RING@@

__device__ __forceinline__ unsigned long long hipmr_ld_agent(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void hipmr_st_agent(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long hipmr_ld_sys(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
// every memory access issued so far has completed (and the compiler moves no
// memory access across this point)
__device__ __forceinline__ void hipmr_drain() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// A job descriptor moved as eight 64-bit words with device-scope accesses.
__device__ __forceinline__ hipmr_sjob hipmr_job_ld(const hipmr_sjob* p, bool system) {
  const unsigned long long* w = (const unsigned long long*)p;
  unsigned long long v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = system ? hipmr_ld_sys(w + k) : hipmr_ld_agent(w + k);
  // every lane read the same words: keep them in scalar registers
#pragma unroll
  for (int k = 0; k < 8; ++k)
    v[k] = (unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v[k] >> 32)) << 32 |
           (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v[k]);
  hipmr_sjob J;
  __builtin_memcpy(&J, v, sizeof(J));
  return J;
}
__device__ __forceinline__ void hipmr_job_st(hipmr_sjob* p, const hipmr_sjob& J) {
  unsigned long long v[8];
  __builtin_memcpy(v, &J, sizeof(J));
#pragma unroll
  for (int k = 0; k < 8; ++k) hipmr_st_agent((unsigned long long*)p + k, v[k]);
}

__device__ __forceinline__ int hipmr_job_ntiles(const hipmr_sjob& J) {
  const int t = hipmr_job_geom(J).tiles;
  return t < 1 ? 1 : t;                 // an empty job still has one (empty) tile
}

#define HIPMR_PUB_TILES(v) ((v) & ((1ull << 40) - 1))
#define HIPMR_MAX_POLLS (1ull << 25)   // polls per wait, whatever the clock says
#define HIPMR_PUB_JOBS(v) ((v) >> 40)

#define HIPMR_RING_WORDS @@RING_WORDS@@            // words per host ring slot (nine used)
#define HIPMR_FIELD ((1ull << 48) - 1)

__device__ __forceinline__ unsigned long long hipmr_ring_tag(unsigned long long s) {
  return ((s / HIPMR_RING) + 1) & 0xffffull;
}

__device__ void hipmr_res_dispatch(unsigned long long* hdr, const unsigned long long* __restrict__ hr_words,
                                   unsigned long long* ctrl, hipmr_sjob* dring,
                                   unsigned long long* dtstart, unsigned long long job_base,
                                   unsigned long long tile_base, unsigned long long epoch,
                                   unsigned long long deadline) {
  const int lane = threadIdx.x & 63;
  const unsigned long long t0 = wall_clock64();
  unsigned long long seq = job_base, stop_at = ~0ull;
  bool closing = false;
  // lanes 0..62 read word lane % 9 of slot seq + lane / 9 (seven slots per
  // read), lane 63 the stop word: one trip over PCIe per pass
  const int js = lane / 9, jw = lane % 9;
  // a second bound besides the clock: every pass takes at least one read of
  // host memory (about a microsecond)
  for (unsigned long long iter = 0;; ++iter) {
    if (!closing) {
      const unsigned long long v =
          lane < 63 ? hipmr_ld_sys(hr_words + ((seq + js) & (HIPMR_RING - 1)) * HIPMR_RING_WORDS + jw)
                    : hipmr_ld_sys(hdr + 16);
      const unsigned long long Sw = hipmr_readlane64(v, 63);
      // the stop word names the instance it is for (epoch << 44 | job index)
      const unsigned long long S = (Sw >> 44) == (epoch & ((1ull << 20) - 1)) ? (Sw & ((1ull << 44) - 1))
                                                                             : ~0ull;
      const unsigned long long m = __ballot(lane < 63 && (v >> 48) == hipmr_ring_tag(seq + js));
      // the instance each job was written for (word 5, bits 32..47): a job
      // of another instance ends this one's jobs, whatever the order in
      // which the reads above saw the ring and the stop word
      const unsigned long long mine =
          __ballot(lane < 63 && jw == 5 && ((v >> 32) & 0xffffull) == (epoch & 0xffffull));
      int cnt = 0;                                     // complete slots of this instance from seq on
      bool other = false;                              // the next complete slot is another instance's
      while (cnt < 7 && ((m >> (9 * cnt)) & 0x1ffull) == 0x1ffull) {
        if (!((mine >> (9 * cnt + 5)) & 1ull)) {
          other = true;
          break;
        }
        ++cnt;
      }
      if (S > seq && (unsigned long long)cnt > S - seq) cnt = (int)(S - seq);
      if (S <= seq) cnt = 0;
      if (cnt > 0) {
        unsigned long long f[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) f[k] = __shfl(v & HIPMR_FIELD, 9 * (lane < cnt ? lane : 0) + k, 64);
        unsigned long long tend = 0;
        if (lane < cnt) {
          const unsigned long long slot = (seq + lane) & (HIPMR_RING - 1);
          hipmr_sjob J;
          J.x = (const void*)f[0];
          J.y = (const void*)f[1];
          J.w = (const void*)f[2];
          J.n = (long long)f[3];
          J.out = (double*)f[4];
          J.tmpl = (int)(f[5] & 0xff);
          J.dtype = (int)((f[5] >> 8) & 0xff);
          J.head = (int)(short)(unsigned short)((f[5] >> 16) & 0xffff);   // signed: -1 = no common alignment
          J.tile0 = 0;
          J.a = __uint_as_float((unsigned)f[6]);
          J.b = __uint_as_float((unsigned)f[7]);
          hipmr_job_st(dring + slot, J);
          hipmr_st_agent(dtstart + slot, f[8]);
          tend = f[8] + (unsigned long long)hipmr_job_ntiles(J);
        }
        tend = hipmr_readlane64(tend, cnt - 1);
        seq += cnt;
        hipmr_drain();                                   // the ring entries are written
        if (lane < 8)
          hipmr_st_agent(ctrl + 32 + 16 * lane, ((seq - job_base) << 40) | (tend - tile_base));
        continue;
      }
      if (S <= seq || other) {
        closing = true;
        stop_at = seq;
      }
    }
    const bool drained = closing && hipmr_ld_agent(ctrl + 16) == stop_at - job_base;
    if (drained || wall_clock64() - t0 > deadline || iter > HIPMR_MAX_POLLS) {
      if (lane < 8) hipmr_st_agent(ctrl + 32 + 16 * lane + 2, 1);
      if (lane == 0)
        __hip_atomic_store(hdr + 32, (epoch << 44) | (seq + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      return;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// Level 1 of the fold of group g of a job whose first tile is js, read with
// device-scope loads (the partials of other waves).
__device__ __forceinline__ double2 hipmr_res_group(bool mx, const unsigned long long* tpart,
                                                   unsigned long long js, unsigned long long mask,
                                                   int g, int ntiles, int lane) {
  const int k = 64 * g + lane;
  double2 v = hipmr_fin_neutral(mx);
  if (k < ntiles) {
    const float2 p = __builtin_bit_cast(float2, hipmr_ld_agent(tpart + ((js + (unsigned long long)k) & mask)));
    v = make_double2((double)p.x, (double)p.y);
  }
  return hipmr_fin_wave(mx, v);
}

extern "C" __global__ void __launch_bounds__(1024)
@@PREFIX@@_res(unsigned long long* hdr, const unsigned long long* __restrict__ hr_words,
               unsigned long long* hr_flags,
               unsigned long long* ctrl, hipmr_sjob* dring, unsigned long long* dtstart,
               unsigned int* gdone, unsigned int* jdone, double2* gpart, float2* tpart_f,
               unsigned long long tp_mask, unsigned long long job_base, unsigned long long tile_base,
               unsigned long long epoch, unsigned long long deadline)
{
  if (blockIdx.x == 0) {
    if (threadIdx.x < 64)
      hipmr_res_dispatch(hdr, hr_words, ctrl, dring, dtstart, job_base, tile_base, epoch, deadline);
    return;
  }
  unsigned long long* tpart = (unsigned long long*)tpart_f;
  unsigned long long* gpw = (unsigned long long*)gpart;      // group values, two words each
  __shared__ unsigned long long sh_t0, sh_pub, sh_jobs;
  __shared__ int sh_stop;
  __shared__ unsigned long long sh_seq[16];    // job of each wave's tile this round
  __shared__ unsigned long long sh_js[16];     // that job's first tile
  __shared__ int sh_k[16];                     // its tile index in the job (-1: none)
  __shared__ float2 sh_part[16];               // the tile's partial
  __shared__ int sh_nt[16];                    // the wave's current job: its tiles,
  __shared__ int sh_tm[16];                    // template
  __shared__ unsigned long long sh_out[16];    // and result address
  // the wave index is uniform: a scalar register, not a vector one per lane
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  unsigned long long* rep = ctrl + 32 + 16 * (blockIdx.x & 7);
  const unsigned long long start = wall_clock64();
  // the wave's current job (its tiles are mostly consecutive tickets)
  unsigned long long cs = 0, cjs = 0;
  int cnt = 0;
  hipmr_sjob cJ;
  unsigned long long hint = job_base;       // no tile of this wave lies in an earlier job
  while (true) {
    if (threadIdx.x == 0)
      sh_t0 = __hip_atomic_fetch_add(ctrl, 16ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const unsigned long long t0 = sh_t0;
    unsigned long long done = t0;           // tickets [t0, done) are handled
    while (done < t0 + 16) {
      if (threadIdx.x == 0) {
        unsigned long long v;
        for (unsigned long long iter = 0;; ++iter) {
          v = hipmr_ld_agent(rep);
          if (HIPMR_PUB_TILES(v) > done) break;
          if (hipmr_ld_agent(rep + 2) != 0 || wall_clock64() - start > deadline + deadline / 8 ||
              iter > HIPMR_MAX_POLLS)
            break;
          __builtin_amdgcn_s_sleep(2);
        }
        sh_pub = HIPMR_PUB_TILES(v);
        sh_jobs = job_base + HIPMR_PUB_JOBS(v);
        sh_stop = HIPMR_PUB_TILES(v) <= done;   // stopped (or past the deadline) with nothing new
      }
      __syncthreads();
      if (sh_stop) return;                  // every published tile was completed before the stop
      const unsigned long long pub = sh_pub, njobs = sh_jobs;
      const unsigned long long avail = pub < t0 + 16 ? pub : t0 + 16;
      const unsigned long long T = t0 + w;
      int myk = -1;
      bool stored = false;
      float2 r = make_float2(0.0f, 0.0f);
      if (T >= done && T < avail) {
        const unsigned long long G = tile_base + T, fresh = tile_base + pub;
        if (!(cnt > 0 && cjs <= G && G < cjs + (unsigned long long)cnt)) {
          // the job holding tile G: the last s in [lo, njobs) whose first tile is <= G.  Slots of
          // completed jobs below it may already hold jobs published later, whose first tiles are
          // >= fresh: they count as <= G, which keeps the predicate monotone.
          unsigned long long lo = hint;
          if (njobs > HIPMR_RING && njobs - HIPMR_RING > lo) lo = njobs - HIPMR_RING;
          unsigned long long hi = njobs - 1;
          // the newest job's descriptor (lanes 0..7, a word each) and first
          // tile (lane 8), read alongside the search: under light load the
          // tile is usually the newest job's, which then costs no second trip
          const unsigned long long hi0 = hi, sslot = hi0 & (HIPMR_RING - 1);
          unsigned long long spec = 0;
          if (lane < 9)
            spec = hipmr_ld_agent(lane < 8 ? (const unsigned long long*)(dring + sslot) + lane : dtstart + sslot);
          while (lo < hi) {
            // lane 63 checks the newest job first: under light load the tile is usually its
            const unsigned long long step = (hi - lo + 64) / 64;
            const unsigned long long cand = lane == 63 ? hi : lo + (unsigned long long)lane * step;
            bool pred = false;
            if (cand <= hi) {
              const unsigned long long ts = hipmr_ld_agent(dtstart + (cand & (HIPMR_RING - 1)));
              pred = ts <= G || ts >= fresh;
            }
            const unsigned long long m = __ballot(pred);
            if (m >> 63) {                  // the newest job holds the tile
              lo = hi;
              break;
            }
            // else lanes 0..62 split [lo, hi - 1]; lane 62's share runs to hi - 1
            const unsigned long long m62 = m & ((1ull << 63) - 1);
            const int kk = m62 ? 63 - __builtin_clzll(m62) : 0;
            const unsigned long long nlo = lo + (unsigned long long)kk * step;
            const unsigned long long nhi = kk == 62 ? hi - 1 : nlo + step - 1;
            lo = nlo;
            hi = nhi < hi - 1 ? nhi : hi - 1;
          }
          hint = lo;
          cs = lo;
          if (lo == hi0) {
            unsigned long long v[8];
#pragma unroll
            for (int k2 = 0; k2 < 8; ++k2) v[k2] = hipmr_readlane64(spec, k2);
            __builtin_memcpy(&cJ, v, sizeof(cJ));
            cjs = hipmr_readlane64(spec, 8);
          } else {
            const unsigned long long slot = lo & (HIPMR_RING - 1);
            cjs = hipmr_ld_agent(dtstart + slot);
            cJ = hipmr_job_ld(dring + slot, false);
          }
          cnt = hipmr_job_ntiles(cJ);
          // for the group fold: the wave's current job, as long as the wave
          // keeps it (written only here, read after the barrier)
          if (lane == 0) {
            sh_nt[w] = cnt;
            sh_tm[w] = cJ.tmpl;
            sh_out[w] = (unsigned long long)cJ.out;
          }
        }
        myk = (int)(G - cjs);
        r = hipmr_job_dispatch(cJ, myk, lane);
        // a group whose tiles all fall in this round ([done, avail), the
        // test the group count below makes) is folded from LDS: only the
        // partials of other groups go to global memory
        const int g0 = myk & ~63;
        const unsigned long long gs = cjs + (unsigned long long)g0 - tile_base;
        const int gsz = cnt - g0 < 64 ? cnt - g0 : 64;
        stored = !(gs >= done && gs + (unsigned long long)gsz <= avail);
        if (stored && lane == 0)
          hipmr_st_agent(tpart + (G & tp_mask), __builtin_bit_cast(unsigned long long, r));
      }
      if (lane == 0) {
        sh_seq[w] = cs;
        sh_js[w] = cjs;
        sh_k[w] = myk;
        sh_part[w] = r;
      }
      if (stored) hipmr_drain();            // this wave's partial is written
      __syncthreads();
      if (w == 0) {
        // count the round's tiles into their groups: lane l < 16 stands for
        // wave l's tile; consecutive waves in the same job and group form a
        // run whose first lane adds the run's length
        const int k = lane < 16 ? sh_k[lane] : -1;
        const unsigned long long s = lane < 16 ? sh_seq[lane] : 0;
        const int g = k >= 0 ? k / 64 : -1;
        const int kp = lane >= 1 && lane < 16 ? sh_k[lane - 1] : -1;
        const unsigned long long sp = lane >= 1 && lane < 16 ? sh_seq[lane - 1] : 0;
        const bool head = k >= 0 && !(kp >= 0 && sp == s && kp / 64 == g);
        int run = 0;
        if (head) {
          run = 1;
          for (int l2 = lane + 1; l2 < 16; ++l2) {
            const int k2 = sh_k[l2];
            if (k2 < 0 || sh_seq[l2] != s || k2 / 64 != g) break;
            ++run;
          }
        }
        bool full = false, local = false;
        if (head) {
          const unsigned long long slot = s & (HIPMR_RING - 1);
          const int ntiles_h = sh_nt[lane];       // the job's tiles, as the wave read them
          const int gsize = ntiles_h - 64 * g < 64 ? ntiles_h - 64 * g : 64;
          if (run == gsize) {
            // the whole group is in this round: no other block holds any of its tiles
            full = local = true;
          } else {
            const unsigned int old = __hip_atomic_fetch_add(gdone + slot * 128 + g, (unsigned)run,
                                                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            full = old + (unsigned)run == (unsigned)gsize;
            if (full)                       // ready for the slot's next job
              __hip_atomic_store(gdone + slot * 128 + g, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
        // fold every group this round completed, one at a time
        unsigned long long todo = __ballot(full);
        while (todo) {
          const int hl = __builtin_ctzll(todo);
          todo &= todo - 1;
          const unsigned long long fs = hipmr_readlane64(s, hl);
          const int fg = __builtin_amdgcn_readlane(g, hl);
          const bool flocal = __builtin_amdgcn_readlane((int)local, hl) != 0;
          const unsigned long long slot = fs & (HIPMR_RING - 1);
          const unsigned long long js = sh_js[hl];
          const int ntiles = sh_nt[hl], ng = (ntiles + 63) / 64, tmpl = sh_tm[hl];
          const bool mx = tmpl == 3;
          double2 gv;
          if (flocal) {                     // the group's partials are this block's: from LDS
            const int gsize = ntiles - 64 * fg < 64 ? ntiles - 64 * fg : 64;
            double2 v = hipmr_fin_neutral(mx);
            if (lane < gsize) {
              const float2 p2 = sh_part[hl + lane];
              v = make_double2((double)p2.x, (double)p2.y);
            }
            gv = hipmr_fin_wave(mx, v);
          } else {
            gv = hipmr_res_group(mx, tpart, js, tp_mask, fg, ntiles, lane);
          }
          bool last = ng == 1;
          double2 tot = gv;
          if (ng == 1) {
            // level 2 over one group: only lane 0 holds a value, and folding
            // the neutral elements of the other lanes into it changes no bit
            tot = hipmr_fin_comb(mx, hipmr_fin_neutral(mx), gv);
          } else {
            if (lane == 0) {
              hipmr_st_agent(gpw + 2 * (slot * 128 + fg), __builtin_bit_cast(unsigned long long, gv.x));
              hipmr_st_agent(gpw + 2 * (slot * 128 + fg) + 1, __builtin_bit_cast(unsigned long long, gv.y));
            }
            hipmr_drain();                  // the group value is written
            unsigned int o2 = 0;
            if (lane == 0) {
              o2 = __hip_atomic_fetch_add(jdone + slot, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              if (o2 + 1 == (unsigned)ng)
                __hip_atomic_store(jdone + slot, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            o2 = __builtin_amdgcn_readlane(o2, 0);
            last = o2 + 1 == (unsigned)ng;
            if (last) {
              const bool h0 = lane < ng, h1 = lane + 64 < ng;
              double2 v0 = make_double2(0.0, 0.0), v1 = v0;
              if (h0) {
                const unsigned long long* q = gpw + 2 * (slot * 128 + lane);
                v0 = make_double2(__builtin_bit_cast(double, hipmr_ld_agent(q)),
                                  __builtin_bit_cast(double, hipmr_ld_agent(q + 1)));
              }
              if (h1) {
                const unsigned long long* q = gpw + 2 * (slot * 128 + lane + 64);
                v1 = make_double2(__builtin_bit_cast(double, hipmr_ld_agent(q)),
                                  __builtin_bit_cast(double, hipmr_ld_agent(q + 1)));
              }
              tot = hipmr_fin_level2(mx, h0, v0, h1, v1);
            }
          }
          if (last && lane == 0) {
            hipmr_job_post_to(tmpl, (double*)sh_out[hl], tot, hr_flags + slot, fs + 1);
            __hip_atomic_fetch_add(ctrl + 16, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
      }
      done = avail;
      __syncthreads();
    }
  }
}
)HIP";

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch()).count();
}

int tile_elems(int32_t dtype) { return dtype == HIPMR_BF16 ? 64 * 8 * 4 : 64 * 4 * 4; }

bool needs_y(int32_t tmpl) { return tmpl == HIPMR_JOB_DOT || tmpl == HIPMR_JOB_AXPBY_SUM; }
bool needs_w(int32_t tmpl) { return tmpl == HIPMR_JOB_WMEAN; }

// Element offset at which all of the job's arrays are 16-byte aligned, or -1.
int job_head(const hipmr_sjob& j) {
    const uintptr_t es = j.dtype == HIPMR_BF16 ? 2 : 4;
    const int vec = (int)(16 / es);
    const void* ptrs[3] = {j.x, needs_y(j.tmpl) ? j.y : nullptr, needs_w(j.tmpl) ? j.w : nullptr};
    for (int h = 0; h < vec; ++h) {
        bool ok = true;
        for (const void* p : ptrs) {
            if (!p) continue;
            uintptr_t a = (uintptr_t)p;
            if (a % es != 0 || (a + h * es) % 16 != 0) ok = false;
        }
        if (ok) return h;
    }
    return -1;
}

// Tiles of a job; the same geometry as hipmr_job_geom in the kernels.
int job_tiles(const hipmr_sjob& j, int head) {
    if (j.n <= 0) return 0;
    const long long tt0 = tile_elems(j.dtype);
    const long long ab = head >= 0 ? std::min<long long>(head, j.n) : 0;
    const long long body = j.n - ab;
    const long long ch = tt0 / 4;                 // one chunk per lane
    const long long c1 = (body + ch - 1) / ch;
    const long long q = c1 > 4 * kRoundTiles ? (c1 + kRoundTiles - 1) / kRoundTiles : 4;
    const long long t = (body + ch * q - 1) / (ch * q);
    return (int)std::max<long long>(t, 1);
}

uint64_t job_bytes(const hipmr_sjob& j) {
    const uint64_t es = j.dtype == HIPMR_BF16 ? 2 : 4;
    const uint64_t arrays = 1 + (needs_y(j.tmpl) ? 1 : 0) + (needs_w(j.tmpl) ? 1 : 0);
    return (uint64_t)std::max<int64_t>(j.n, 0) * es * arrays + 8;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Device workspace of the resident mode: control words, the device copy of
// the descriptor ring and the first tile of each, per slot 128 group counters
// and group values, per slot a job counter, and the ring of tile partials.
struct ResLayout {
    size_t ctrl, dring, dtstart, gdone, jdone, gpart, tpart, total;
    uint64_t tp;          // tile partials (a power of two >= max_batch_tiles)
};

ResLayout res_layout(const hipmr_server_config& c) {
    ResLayout L{};
    uint64_t tp = 8192;
    while (tp < (uint64_t)c.max_batch_tiles) tp <<= 1;
    L.tp = tp;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off += (bytes + 255) & ~size_t(255);
        return at;
    };
    L.ctrl = take(kCtrlBytes);
    L.dring = take((size_t)kRing * sizeof(DevJob));
    L.dtstart = take((size_t)kRing * 8);
    L.gdone = take((size_t)kRing * 128 * 4);
    L.jdone = take((size_t)kRing * 4);
    L.gpart = take((size_t)kRing * 128 * 16);
    L.tpart = take((size_t)tp * 8);
    L.total = off;
    return L;
}

size_t slot_bytes(const hipmr_server_config& c) {
    return align256((size_t)c.max_batch_jobs * sizeof(DevJob)) + align256((size_t)c.max_batch_tiles * 8);
}

hipmr_server_config resolved(const hipmr_server_config* in) {
    hipmr_server_config c{};
    if (in) c = *in;
    if (c.hbm_budget_bytes == 0) c.hbm_budget_bytes = 64ull << 30;
    if (c.nstreams == 0) c.nstreams = 4;
    if (c.max_batch_jobs == 0) c.max_batch_jobs = 1024;
    if (c.max_batch_tiles == 0) c.max_batch_tiles = 1 << 18;
    if (c.max_batch_bytes == 0) c.max_batch_bytes = 16ull << 20;
    if (c.solo_bytes == 0) c.solo_bytes = std::min<uint64_t>(4ull << 20, c.max_batch_bytes);
    if (c.batch_backlog == 0) c.batch_backlog = 8;
    if (c.resident && c.blocks_per_cu == 0) c.blocks_per_cu = 1;
    if (c.blocks_per_cu == 0) c.blocks_per_cu = 8;
    return c;
}

}  // namespace

namespace hipmr {

// Device source of the serving kernels, specialised by keyword replacement.
std::string serve_source(const std::string& prefix) {
    std::string src = std::string("// generated by hipmr: serving kernels\n") + device_prelude() + kServeKernels;
    auto rep = [&](const std::string& key, const std::string& val) {
        size_t pos = 0;
        while ((pos = src.find(key, pos)) != std::string::npos) {
            src.replace(pos, key.size(), val);
            pos += val.size();
        }
    };
    rep("@@PREFIX@@", prefix);
    rep("@@BF16CODE@@", std::to_string(HIPMR_BF16));
    rep("@@ROUND_TILES@@", std::to_string(kRoundTiles));
    rep("@@NINLINE@@", std::to_string(kInlineJobs));
    rep("@@RING@@", std::to_string(kRing));
    rep("@@RING_WORDS@@", std::to_string(kRingWords));
    return src;
}

}  // namespace hipmr

struct hipmr_server {
    hipmr_server_config cfg{};
    int device = 0;
    std::shared_ptr<CodeObject> co;
    hipModule_t module = nullptr;
    hipFunction_t f_s1 = nullptr, f_s2 = nullptr, f_one1 = nullptr, f_one2 = nullptr;
    hipFunction_t f_i1 = nullptr, f_i2 = nullptr, f_one = nullptr, f_res = nullptr;
    std::string prefix;
    int cus = 256;


    struct Pending {
        hipmr_sjob job;
        uint64_t ticket;
        int64_t arrival_ns;
        uint64_t bytes;
        int tiles;
        int head;
    };
    // resident mode: the host ring (mapped host memory), the device workspace
    // parts, and the state of the instance on the device
    struct Res {
        hipStream_t stream = nullptr;
        uint64_t* hdr = nullptr;            // host view; [16] stop word, [32] exit word
        uint64_t* words = nullptr;          // kRing slots of kRingWords tagged words
        uint64_t* flags = nullptr;
        void *hdr_d = nullptr, *words_d = nullptr, *flags_d = nullptr;
        char* ws = nullptr;
        ResLayout L{};
        int grid = 0;
        uint64_t deadline_ticks = 0;
        uint64_t next_seq = 0, next_tile = 0, epoch = 0;
        bool running = false;
        int64_t launched_ns = 0, last_busy_ns = 0, last_query_ns = 0;
        struct Flight {
            Pending p;
            uint64_t seq, tile0, tiles;
            int64_t published_ns;
            int32_t on_device;
        };
        std::deque<Flight> flights;         // published, not completed, in publish order
    } res;
    struct Slot {
        hipStream_t stream = nullptr;
        DevJob* host_desc = nullptr;    // pinned host memory
        uint64_t* flags = nullptr;      // per-job completion flags (host memory, mapped)
        uint64_t* dev_flags = nullptr;  // the same memory, as the device sees it
        uint64_t seq = 0;               // the current batch's flag value
        DevJob* dev_desc = nullptr;     // in the caller's workspace
        void* tpart = nullptr;          // in the caller's workspace
        std::vector<Pending> jobs;
        int64_t launch_ns = 0;
        bool busy = false;
    };
    std::vector<Slot> slots;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Pending> incoming;       // submitted, not yet seen by the loop
    std::deque<Pending> waiting;        // arrived, not yet admitted (loop thread only)
    std::vector<Pending> skipped;       // large jobs a batch of small ones was packed past
    std::vector<hipmr_completion> finished;   // for poll
    uint64_t next_ticket = 1;
    uint64_t admitted = 0;              // bytes of admitted, unfinished jobs
    int64_t unfinished = 0;             // submitted, not completed

    // open-loop schedule replay
    const hipmr_sjob* sched = nullptr;
    int32_t sched_n = 0, sched_next = 0, sched_done = 0;
    int64_t sched_t0 = 0;
    hipmr_completion* sched_out = nullptr;

    std::atomic<bool> stop{false};
    hipmr_status worker_status = HIPMR_OK;
    std::string worker_error;
    std::thread worker;

    // Frees what hipmr_server_create allocated, also when it failed part
    // way; runs after the loop's thread has ended (or was never started).
    ~hipmr_server() {
        if (res.stream) {
            // the instance reads the host ring until it exits: stop it (if the
            // loop did not) and wait before the ring is freed
            if (res.running && res.hdr) stop_instance();
            (void)hipStreamSynchronize(res.stream);
            (void)hipStreamDestroy(res.stream);
        }
        if (res.hdr) (void)hipHostFree(res.hdr);
        for (auto& sl : slots) {
            if (sl.stream) (void)hipStreamSynchronize(sl.stream);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
            if (sl.host_desc) (void)hipHostFree(sl.host_desc);
            if (sl.flags) (void)hipHostFree(sl.flags);
        }
        if (module) (void)hipModuleUnload(module);
    }

    void complete(const Pending& p, int32_t status, int32_t batch_jobs, int64_t launch, int64_t done) {
        hipmr_completion c{};
        c.ticket = p.ticket;
        c.status = status;
        c.batch_jobs = batch_jobs;
        c.arrival_ns = p.arrival_ns;
        c.launch_ns = launch;
        c.done_ns = done;
        std::lock_guard<std::mutex> lk(mu);
        if (sched_out && p.ticket >= 1ull << 62) {
            sched_out[p.ticket - (1ull << 62)] = c;
            ++sched_done;
        } else {
            finished.push_back(c);
        }
        --unfinished;
        cv_done.notify_all();
    }

    hipmr_status launch_batch(Slot& s) {
        const int nj = (int)s.jobs.size();
        ++s.seq;
        if (nj == 1 && cfg.max_batch_jobs > 1 && s.jobs[0].tiles <= kOneLaunchTiles) {
            // a small job alone: one launch (the one-launch-pair-per-job
            // baseline, max_batch_jobs = 1, keeps its two)
            const Pending& p = s.jobs[0];
            DevJob d{p.job.x, p.job.y, p.job.w, p.job.n, p.job.tmpl, p.job.dtype, 0, p.head,
                     p.job.out, p.job.a, p.job.b};
            void* a[4] = {&d, &s.tpart, &s.dev_flags, &s.seq};
            hipError_t e = hipModuleLaunchKernel(f_one, 1, 1, 1, kFinBlock, 1, 1, 0, s.stream, a, nullptr);
            if (e != hipSuccess) return fail(HIPMR_E_HIP, std::string("serving launch: ") + hipGetErrorString(e));
        } else if (nj == 1) {       // one job: its descriptor by value
            const Pending& p = s.jobs[0];
            DevJob d{p.job.x, p.job.y, p.job.w, p.job.n, p.job.tmpl, p.job.dtype, 0, p.head,
                     p.job.out, p.job.a, p.job.b};
            int grid = std::max(1, std::min(cfg.blocks_per_cu * cus, (p.tiles + 3) / 4));
            void* a1[2] = {&d, &s.tpart};
            hipError_t e = hipModuleLaunchKernel(f_one1, grid, 1, 1, kServeBlock, 1, 1, 0, s.stream, a1, nullptr);
            if (e == hipSuccess) {
                void* a2[4] = {&d, &s.tpart, &s.dev_flags, &s.seq};
                e = hipModuleLaunchKernel(f_one2, 1, 1, 1, kFinBlock, 1, 1, 0, s.stream, a2, nullptr);
            }
            if (e != hipSuccess) return fail(HIPMR_E_HIP, std::string("serving launch: ") + hipGetErrorString(e));
        } else if (nj <= kInlineJobs) {
            InlineJobs b{};
            int tile0 = 0;
            for (int k = 0; k < nj; ++k) {
                const Pending& p = s.jobs[k];
                b.jobs[k] = DevJob{p.job.x, p.job.y, p.job.w, p.job.n, p.job.tmpl, p.job.dtype,
                                   tile0, p.head, p.job.out, p.job.a, p.job.b};
                tile0 += p.tiles;
            }
            b.njobs = nj;
            b.total_tiles = tile0;
            int grid = std::max(1, std::min(cfg.blocks_per_cu * cus, (tile0 + 3) / 4));
            void* a1[2] = {&b, &s.tpart};
            hipError_t e = hipModuleLaunchKernel(f_i1, grid, 1, 1, kServeBlock, 1, 1, 0, s.stream, a1, nullptr);
            void* a2[4] = {&b, &s.tpart, &s.dev_flags, &s.seq};
            if (e == hipSuccess)
                e = hipModuleLaunchKernel(f_i2, nj, 1, 1, kFinBlock, 1, 1, 0, s.stream, a2, nullptr);
            if (e != hipSuccess) return fail(HIPMR_E_HIP, std::string("serving launch: ") + hipGetErrorString(e));
        } else {
            int tile0 = 0;
            for (int k = 0; k < nj; ++k) {
                const Pending& p = s.jobs[k];
                s.host_desc[k] = DevJob{p.job.x, p.job.y, p.job.w, p.job.n, p.job.tmpl, p.job.dtype,
                                        tile0, p.head, p.job.out, p.job.a, p.job.b};
                tile0 += p.tiles;
            }
            int total = tile0;
            hipError_t e = hipMemcpyAsync(s.dev_desc, s.host_desc, (size_t)nj * sizeof(DevJob),
                                          hipMemcpyHostToDevice, s.stream);
            int grid = std::max(1, std::min(cfg.blocks_per_cu * cus, (total + 3) / 4));
            void* a1[4] = {&s.dev_desc, (void*)&nj, &total, &s.tpart};
            if (e == hipSuccess)
                e = hipModuleLaunchKernel(f_s1, grid, 1, 1, kServeBlock, 1, 1, (unsigned)nj * 4, s.stream,
                                          a1, nullptr);
            void* a2[6] = {&s.dev_desc, (void*)&nj, &total, &s.tpart, &s.dev_flags, &s.seq};
            if (e == hipSuccess)
                e = hipModuleLaunchKernel(f_s2, nj, 1, 1, kFinBlock, 1, 1, 0, s.stream, a2, nullptr);
            if (e != hipSuccess) return fail(HIPMR_E_HIP, std::string("serving launch: ") + hipGetErrorString(e));
        }
        s.launch_ns = now_ns();
        s.busy = true;
        return HIPMR_OK;
    }

    // ------------------------------------------------------------ resident
    // Stops the running instance at the next job index: it finishes the jobs
    // it accepted and exits.
    void stop_instance() {
        __atomic_store_n(&res.hdr[16], (res.epoch << kEpochShift) | res.next_seq, __ATOMIC_RELEASE);
        res.running = false;
    }

    // Launches an instance that takes the jobs from res.next_seq on; it runs
    // after the previous instance (same stream) has exited.
    hipmr_status launch_instance() {
        ++res.epoch;
        char* w = res.ws;
        void* ctrl = w + res.L.ctrl;
        hipError_t e = hipMemsetAsync(ctrl, 0, kCtrlBytes, res.stream);
        void* dring = w + res.L.dring;
        void* dtstart = w + res.L.dtstart;
        void* gdone = w + res.L.gdone;
        void* jdone = w + res.L.jdone;
        void* gpart = w + res.L.gpart;
        void* tpart = w + res.L.tpart;
        unsigned long long mask = res.L.tp - 1, jb = res.next_seq, tb = res.next_tile, ep = res.epoch,
                           dl = res.deadline_ticks;
        void* a[15] = {&res.hdr_d, &res.words_d, &res.flags_d, &ctrl, &dring, &dtstart,
                       &gdone, &jdone, &gpart, &tpart, &mask, &jb, &tb, &ep, &dl};
        if (e == hipSuccess)
            e = hipModuleLaunchKernel(f_res, (unsigned)res.grid, 1, 1, 1024, 1, 1, 0, res.stream, a, nullptr);
        if (e != hipSuccess)
            return fail(HIPMR_E_HIP, std::string("resident launch: ") + hipGetErrorString(e));
        res.running = true;
        res.launched_ns = now_ns();
        return HIPMR_OK;
    }

    void fail_flights(hipmr_status st) {
        const int64_t t = now_ns();
        for (const auto& f : res.flights) {
            admitted -= f.p.bytes;
            complete(f.p, st, f.on_device, f.published_ns, t);
        }
        res.flights.clear();
    }

    bool step_resident() {
        bool progressed = take_arrivals();
        const int64_t t = now_ns();
        // completions: each job's flag holds its index + 1 once its result is written
        for (auto it = res.flights.begin(); it != res.flights.end();) {
            if (*(volatile uint64_t*)&res.flags[it->seq & (kRing - 1)] == it->seq + 1) {
                admitted -= it->p.bytes;
                complete(it->p, HIPMR_OK, it->on_device, it->published_ns, now_ns());
                it = res.flights.erase(it);
                progressed = true;
            } else {
                ++it;
            }
        }
        // watchdog: errors of the stream, and jobs the instance can no longer finish
        if (!res.flights.empty() && t - res.flights.front().published_ns > kWatchdogNs &&
            t - res.last_query_ns > kWatchdogNs) {
            res.last_query_ns = t;
            hipError_t q = hipStreamQuery(res.stream);
            const bool late = t - res.flights.front().published_ns > (int64_t)(2.5 * kLifeS * 1e9);
            if ((q != hipSuccess && q != hipErrorNotReady) || late) {
                std::lock_guard<std::mutex> lk(mu);
                worker_status = HIPMR_E_HIP;
                worker_error = q != hipSuccess && q != hipErrorNotReady
                                   ? std::string("resident kernel: ") + hipGetErrorString(q)
                                   : "resident kernel: jobs not completed by the instance's deadline";
            }
            if ((q != hipSuccess && q != hipErrorNotReady) || late) {
                fail_flights(HIPMR_E_HIP);
                if (res.running) stop_instance();
                progressed = true;
            }
        }
        // admission: in arrival order while the budget, the descriptor ring and
        // the ring of tile partials have room
        while (!waiting.empty()) {
            const Pending& p = waiting.front();
            const uint64_t tiles = (uint64_t)std::max(1, p.tiles);
            const uint64_t oldest_seq = res.flights.empty() ? res.next_seq : res.flights.front().seq;
            const uint64_t oldest_tile = res.flights.empty() ? res.next_tile : res.flights.front().tile0;
            if (admitted + p.bytes > cfg.hbm_budget_bytes) break;
            if (res.next_seq - oldest_seq >= (uint64_t)kRing) break;
            if (res.next_tile + tiles - oldest_tile > res.L.tp) break;
            if (!res.running) {
                hipmr_status st = launch_instance();
                if (st != HIPMR_OK) {
                    {
                        std::lock_guard<std::mutex> lk(mu);
                        worker_status = st;
                        worker_error = last_error();
                    }
                    complete(p, st, 0, t, now_ns());
                    waiting.pop_front();
                    progressed = true;
                    continue;
                }
            }
            // the nine tagged words of the job's slot (their order does not
            // matter: the device takes the slot once all nine carry the tag)
            const uint64_t slot = res.next_seq & (kRing - 1);
            const uint64_t tag = ((res.next_seq / kRing + 1) & 0xffff) << 48;
            uint32_t ab[2];
            std::memcpy(&ab[0], &p.job.a, 4);
            std::memcpy(&ab[1], &p.job.b, 4);
            const uint64_t f[9] = {(uint64_t)(uintptr_t)p.job.x, (uint64_t)(uintptr_t)p.job.y,
                                   (uint64_t)(uintptr_t)p.job.w, (uint64_t)p.job.n,
                                   (uint64_t)(uintptr_t)p.job.out,
                                   (uint64_t)p.job.tmpl | ((uint64_t)p.job.dtype << 8) |
                                       ((uint64_t)(uint16_t)(int16_t)p.head << 16) |   // head: -1 or 0..7
                                       ((res.epoch & 0xffff) << 32),                    // the instance's
                                   ab[0], ab[1], res.next_tile};
            uint64_t* dst = res.words + slot * kRingWords;
            for (int k = 0; k < 9; ++k) __atomic_store_n(dst + k, tag | (f[k] & kField), __ATOMIC_RELEASE);
            res.flights.push_back({p, res.next_seq, res.next_tile, tiles, now_ns(),
                                   (int32_t)res.flights.size() + 1});
            admitted += p.bytes;
            ++res.next_seq;
            res.next_tile += tiles;
            waiting.pop_front();
            progressed = true;
        }
        // the instance: a new one every kRotateNs (so none reaches its
        // deadline), none while idle for kIdleStopNs
        const int64_t t2 = now_ns();
        if (!res.flights.empty() || !waiting.empty()) res.last_busy_ns = t2;
        if (res.running) {
            if (t2 - res.last_busy_ns > kIdleStopNs) {
                stop_instance();
            } else if (t2 - res.launched_ns > kRotateNs) {
                stop_instance();
                hipmr_status st = launch_instance();
                if (st != HIPMR_OK) {
                    std::lock_guard<std::mutex> lk(mu);
                    worker_status = st;
                    worker_error = last_error();
                }
            }
        }
        return progressed;
    }

    // Arrivals: submitted jobs and scheduled jobs whose time has come join
    // the waiting queue.
    bool take_arrivals() {
        bool progressed = false;
        const int64_t t = now_ns();
        std::lock_guard<std::mutex> lk(mu);
        while (!incoming.empty()) {
            waiting.push_back(incoming.front());
            incoming.pop_front();
            progressed = true;
        }
        while (sched && sched_next < sched_n && sched_t0 + sched[sched_next].arrival_ns <= t) {
            const hipmr_sjob& j = sched[sched_next];
            Pending p{j, (1ull << 62) + (uint64_t)sched_next, sched_t0 + j.arrival_ns, job_bytes(j), 0,
                      job_head(j)};
            p.tiles = job_tiles(j, p.head);
            waiting.push_back(p);
            ++sched_next;
            progressed = true;
        }
        return progressed;
    }

    // One pass of the loop; returns true if it did anything.
    bool step() {
        if (cfg.resident) return step_resident();
        bool progressed = take_arrivals();
        // completions
        for (Slot& s : slots) {
            if (!s.busy) continue;
            // every job's flag carries this batch's sequence number once its
            // result is written; the stream is queried only as a watchdog for
            // errors
            bool all = true;
            for (size_t k = 0; k < s.jobs.size() && all; ++k)
                all = *(volatile uint64_t*)&s.flags[k] == s.seq;
            int32_t st = HIPMR_OK;
            if (!all) {
                if (now_ns() - s.launch_ns < kWatchdogNs) continue;
                hipError_t q = hipStreamQuery(s.stream);
                if (q == hipErrorNotReady) continue;
                all = true;
                for (size_t k = 0; k < s.jobs.size() && all; ++k)
                    all = *(volatile uint64_t*)&s.flags[k] == s.seq;
                if (q != hipSuccess || !all) st = HIPMR_E_HIP;
            }
            const int64_t done = now_ns();
            for (const Pending& p : s.jobs) {
                admitted -= p.bytes;
                complete(p, st, (int32_t)s.jobs.size(), s.launch_ns, done);
            }
            s.jobs.clear();
            s.busy = false;
            progressed = true;
        }
        // admission + packing into free slots.  While at most batch_backlog
        // jobs per free slot wait, each free slot takes one job, as the
        // one-launch-pair-per-job loop would (packing a short queue into one
        // stream measured a longer p99 than spreading it); a longer queue is
        // spread over the free slots, ceil(waiting / free) jobs per batch, so
        // batches grow with the backlog and drain it.  A job of more than
        // solo_bytes runs in a batch of its own; a batch of smaller jobs is
        // packed past such jobs, which stay queued (not yet admitted) for the
        // next free slot, so a small job never waits for a large one's tiles.
        // Packing stops at the first job, skipped or not, that does not fit
        // the budget: no job is admitted while an earlier one does not fit.
        int free_slots = 0;
        for (const Slot& s : slots) free_slots += !s.busy;
        for (Slot& s : slots) {
            if (s.busy || waiting.empty()) continue;
            const size_t w = waiting.size();
            const size_t quota = w <= (size_t)cfg.batch_backlog * free_slots ? 1 : (w + free_slots - 1) / free_slots;
            --free_slots;
            if (waiting.front().bytes > cfg.solo_bytes) {
                const Pending& p = waiting.front();
                if (admitted + p.bytes > cfg.hbm_budget_bytes) break;
                admitted += p.bytes;
                s.jobs.push_back(p);
                waiting.pop_front();
            } else {
                int tiles = 0;
                uint64_t bytes = 0;
                skipped.clear();
                while (!waiting.empty() && (int)s.jobs.size() < cfg.max_batch_jobs &&
                       s.jobs.size() < quota) {
                    const Pending& p = waiting.front();
                    if (admitted + p.bytes > cfg.hbm_budget_bytes) break;
                    if (p.bytes > cfg.solo_bytes) {
                        if ((int)skipped.size() == kMaxSkipped) break;
                        skipped.push_back(p);
                        waiting.pop_front();
                        continue;
                    }
                    if (!s.jobs.empty() &&
                        (tiles + p.tiles > cfg.max_batch_tiles || bytes + p.bytes > cfg.max_batch_bytes))
                        break;
                    admitted += p.bytes;
                    tiles += p.tiles;
                    bytes += p.bytes;
                    s.jobs.push_back(p);
                    waiting.pop_front();
                }
                for (auto it = skipped.rbegin(); it != skipped.rend(); ++it) waiting.push_front(*it);
            }
            if (s.jobs.empty()) break;       // budget full: wait for completions
            hipmr_status st = launch_batch(s);
            if (st != HIPMR_OK) {
                {
                    std::lock_guard<std::mutex> lk(mu);
                    worker_status = st;
                    worker_error = last_error();
                }
                for (const Pending& p : s.jobs) {
                    admitted -= p.bytes;
                    complete(p, st, (int32_t)s.jobs.size(), now_ns(), now_ns());
                }
                s.jobs.clear();
            }
            progressed = true;
        }
        return progressed;
    }

    // The loop cannot use the device: every job, submitted or scheduled, is
    // completed at once with E_HIP (nothing waits for a result that never
    // comes) until the server is destroyed.
    void fail_every_job() {
        while (true) {
            std::vector<Pending> failed;
            {
                std::unique_lock<std::mutex> lk(mu);
                while (!incoming.empty()) {
                    failed.push_back(incoming.front());
                    incoming.pop_front();
                }
                while (sched && sched_next < sched_n) {
                    const hipmr_sjob& j = sched[sched_next];
                    failed.push_back(Pending{j, (1ull << 62) + (uint64_t)sched_next, sched_t0 + j.arrival_ns,
                                             job_bytes(j), 0, 0});
                    ++sched_next;
                }
                if (failed.empty()) {
                    if (stop.load()) return;
                    cv_work.wait_for(lk, std::chrono::milliseconds(2));
                    continue;
                }
            }
            const int64_t t = now_ns();
            for (const Pending& p : failed) complete(p, HIPMR_E_HIP, 0, t, t);
        }
    }

    void loop() {
        if (hipSetDevice(device) != hipSuccess) {
            {
                std::lock_guard<std::mutex> lk(mu);
                worker_status = HIPMR_E_HIP;
                worker_error = "hipSetDevice failed in the serving thread";
            }
            fail_every_job();
            return;
        }
        while (true) {
            bool progressed = step();
            if (stop.load()) {
                bool busy = !res.flights.empty();
                for (Slot& s : slots) busy |= s.busy;
                std::lock_guard<std::mutex> lk(mu);
                if (!busy && incoming.empty() && waiting.empty()) break;
            }
            if (!progressed) {
                bool busy = !res.flights.empty();
                for (Slot& s : slots) busy |= s.busy;
                std::unique_lock<std::mutex> lk(mu);
                bool sched_pending = sched && sched_next < sched_n;
                if (!busy && waiting.empty() && incoming.empty() && !sched_pending) {
                    cv_work.wait_for(lk, std::chrono::milliseconds(2));
                } else {
                    lk.unlock();
                    std::this_thread::yield();
                }
            }
        }
        if (res.running) stop_instance();
    }
};

namespace {

hipmr_status validate_job(const hipmr_server* s, const hipmr_sjob* j) {
    if (!j) return fail(HIPMR_E_INVALID, "NULL job");
    if (j->tmpl < 0 || j->tmpl > HIPMR_JOB_WMEAN) return fail(HIPMR_E_INVALID, "unknown job template");
    if (j->dtype != HIPMR_F32 && j->dtype != HIPMR_BF16)
        return fail(HIPMR_E_UNSUPPORTED, "serving jobs take float or bfloat16 arrays");
    if (j->n < 0) return fail(HIPMR_E_INVALID, "n must be >= 0");
    if (!j->out) return fail(HIPMR_E_INVALID, "out is NULL");
    if (j->n > 0 && (!j->x || (needs_y(j->tmpl) && !j->y) || (needs_w(j->tmpl) && !j->w)))
        return fail(HIPMR_E_INVALID, "an input array of the job's template is NULL");
    if (job_bytes(*j) > s->cfg.hbm_budget_bytes)
        return fail(HIPMR_E_BUDGET, "the job alone exceeds the memory budget");
    if ((std::max<int64_t>(j->n, 0) + tile_elems(j->dtype) - 1) / tile_elems(j->dtype) > kMaxBaseTiles)
        return fail(HIPMR_E_UNSUPPORTED, "the job is over 2^26 float32 or 2^27 bfloat16 elements");
    if (job_tiles(*j, job_head(*j)) > s->cfg.max_batch_tiles)
        return fail(HIPMR_E_BUDGET, "the job has more tiles than max_batch_tiles");
    if (s->cfg.resident &&
        (((uintptr_t)j->x | (uintptr_t)j->y | (uintptr_t)j->w | (uintptr_t)j->out) > kField ||
         (uint64_t)j->n > kField))
        return fail(HIPMR_E_UNSUPPORTED, "the resident ring carries addresses and lengths below 2^48");
    return HIPMR_OK;
}

}  // namespace

extern "C" {

int64_t hipmr_server_now_ns(void) { return now_ns(); }

size_t hipmr_server_workspace_bytes(const hipmr_server_config* in) {
    hipmr_server_config c = resolved(in);
    if (c.resident) return res_layout(c).total;
    return (size_t)c.nstreams * slot_bytes(c);
}

hipmr_status hipmr_server_create(const hipmr_server_config* in, void* workspace, size_t workspace_bytes,
                                 hipmr_server_t* out) {
    clear_error();
    if (!out) return fail(HIPMR_E_INVALID, "NULL argument");
    *out = nullptr;
    hipmr_server_config c = resolved(in);
    if (c.nstreams < 1 || c.nstreams > 16) return fail(HIPMR_E_INVALID, "nstreams must be in [1, 16]");
    if (c.max_batch_jobs < 1 || c.max_batch_jobs > kMaxBatchJobs)
        return fail(HIPMR_E_INVALID, "max_batch_jobs must be in [1, 4096]");
    if (c.max_batch_tiles < 1 || c.blocks_per_cu < 1) return fail(HIPMR_E_INVALID, "bad batch limits");
    if (c.batch_backlog < 0) return fail(HIPMR_E_INVALID, "batch_backlog must be >= 0");
    if (c.solo_bytes > c.max_batch_bytes)
        return fail(HIPMR_E_INVALID, "solo_bytes must not exceed max_batch_bytes");
    if (!workspace || workspace_bytes < hipmr_server_workspace_bytes(&c))
        return fail(HIPMR_E_WORKSPACE, "workspace smaller than hipmr_server_workspace_bytes()");
    auto s = std::make_unique<hipmr_server>();
    s->cfg = c;
    if (hipGetDevice(&s->device) != hipSuccess) return fail(HIPMR_E_HIP, "hipGetDevice failed");
    s->cus = device_cu_count();
    // compile the serving kernels (templates x dtypes) through the RTC cache
    s->prefix = "hipmr_serve";
    hipmr_status st;
    s->co = get_or_build(serve_source(s->prefix), s->prefix + "_s1", &st);
    if (!s->co) return st;
    const std::string& image = code_object_image(*s->co);
    hipError_t e = hipModuleLoadData(&s->module, image.data());
    if (e != hipSuccess) return fail(HIPMR_E_HIP, std::string("hipModuleLoadData: ") + hipGetErrorString(e));
    struct { hipFunction_t* f; const char* suffix; } fns[] = {
        {&s->f_s1, "_s1"}, {&s->f_s2, "_s2"}, {&s->f_one1, "_one1"}, {&s->f_one2, "_one2"},
        {&s->f_i1, "_i1"}, {&s->f_i2, "_i2"}, {&s->f_one, "_one"}, {&s->f_res, "_res"}};
    for (auto& f : fns) {
        e = hipModuleGetFunction(f.f, s->module, (s->prefix + f.suffix).c_str());
        if (e != hipSuccess) return fail(HIPMR_E_HIP, std::string("hipModuleGetFunction: ") + hipGetErrorString(e));
    }
    if (c.resident) {
        auto& r = s->res;
        r.L = res_layout(c);
        r.ws = (char*)workspace;
        int per_cu = 0, khz = 0;
        if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, s->f_res, 1024, 0) != hipSuccess ||
            per_cu < 1)
            return fail(HIPMR_E_HIP, "the resident kernel does not fit a CU with 1024 threads");
        r.grid = std::min(c.blocks_per_cu, per_cu) * s->cus;
        if (r.grid < 2) return fail(HIPMR_E_HIP, "the resident kernel needs at least two blocks");
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, s->device) != hipSuccess ||
            khz < 1000 || khz > 10000000)
            return fail(HIPMR_E_HIP, "the device wall clock rate is unknown");
        r.deadline_ticks = (uint64_t)(kLifeS * 1e3 * khz);
        const size_t ring = 512 + (size_t)kRing * (kRingWords * 8 + 8);
        // default-priority, non-blocking stream; the ring in mapped, coherent host memory
        if (hipStreamCreateWithFlags(&r.stream, hipStreamNonBlocking) != hipSuccess ||
            hipHostMalloc((void**)&r.hdr, ring, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
            return fail(HIPMR_E_HIP, "creating the resident stream or its host ring failed");
        std::memset(r.hdr, 0, ring);
        r.words = (uint64_t*)((char*)r.hdr + 512);
        r.flags = r.words + (size_t)kRing * kRingWords;
        void* hd = nullptr;
        if (hipHostGetDevicePointer(&hd, r.hdr, 0) != hipSuccess)
            return fail(HIPMR_E_HIP, "hipHostGetDevicePointer failed for the host ring");
        r.hdr_d = hd;
        r.words_d = (char*)hd + 512;
        r.flags_d = (char*)r.words_d + (size_t)kRing * kRingWords * 8;
        // no instance yet: the stop word names epoch 0, which never runs
        r.hdr[16] = 0;
        if (hipMemsetAsync(workspace, 0, r.L.total, r.stream) != hipSuccess ||
            hipStreamSynchronize(r.stream) != hipSuccess)
            return fail(HIPMR_E_HIP, "clearing the resident workspace failed");
        hipmr_server* raw = s.get();
        s->worker = std::thread([raw] { raw->loop(); });
        *out = s.release();
        return HIPMR_OK;
    }
    s->slots.resize(c.nstreams);
    char* base = (char*)workspace;
    for (int k = 0; k < c.nstreams; ++k) {
        auto& sl = s->slots[k];
        // default-priority, non-blocking streams
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipHostMalloc((void**)&sl.host_desc, (size_t)c.max_batch_jobs * sizeof(DevJob),
                          hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&sl.flags, (size_t)c.max_batch_jobs * sizeof(uint64_t),
                          hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
            hipHostGetDevicePointer((void**)&sl.dev_flags, sl.flags, 0) != hipSuccess)
            return fail(HIPMR_E_HIP, "creating the serving streams or pinned buffers failed");
        std::memset(sl.flags, 0, (size_t)c.max_batch_jobs * sizeof(uint64_t));
        sl.dev_desc = (DevJob*)(base + (size_t)k * slot_bytes(c));
        sl.tpart = base + (size_t)k * slot_bytes(c) + align256((size_t)c.max_batch_jobs * sizeof(DevJob));
    }
    hipmr_server* raw = s.get();
    s->worker = std::thread([raw] { raw->loop(); });
    *out = s.release();
    return HIPMR_OK;
}

hipmr_status hipmr_server_submit(hipmr_server_t s, const hipmr_sjob* job, uint64_t* ticket) {
    clear_error();
    if (!s) return fail(HIPMR_E_INVALID, "NULL server");
    hipmr_status st = validate_job(s, job);
    if (st != HIPMR_OK) return st;
    hipmr_server::Pending p{*job, 0, now_ns(), job_bytes(*job), 0, job_head(*job)};
    p.tiles = job_tiles(*job, p.head);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        p.ticket = s->next_ticket++;
        s->incoming.push_back(p);
        ++s->unfinished;
    }
    s->cv_work.notify_one();
    if (ticket) *ticket = p.ticket;
    return HIPMR_OK;
}

hipmr_status hipmr_server_poll(hipmr_server_t s, hipmr_completion* done, int32_t cap, int32_t* ndone) {
    clear_error();
    if (!s || !ndone || (cap > 0 && !done)) return fail(HIPMR_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    const int32_t k = (int32_t)std::min<size_t>((size_t)std::max(cap, 0), s->finished.size());
    std::copy(s->finished.begin(), s->finished.begin() + k, done);
    s->finished.erase(s->finished.begin(), s->finished.begin() + k);
    *ndone = k;
    if (s->worker_status != HIPMR_OK) return fail(s->worker_status, s->worker_error);
    return HIPMR_OK;
}

hipmr_status hipmr_server_wait_idle(hipmr_server_t s) {
    clear_error();
    if (!s) return fail(HIPMR_E_INVALID, "NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->unfinished == 0; });
    return HIPMR_OK;
}

hipmr_status hipmr_server_run_schedule(hipmr_server_t s, const hipmr_sjob* jobs, int32_t njobs,
                                       hipmr_completion* done) {
    clear_error();
    if (!s || (njobs > 0 && (!jobs || !done)) || njobs < 0) return fail(HIPMR_E_INVALID, "NULL argument");
    int32_t valid = 0;
    for (int32_t k = 0; k < njobs; ++k) {
        if (k > 0 && jobs[k].arrival_ns < jobs[k - 1].arrival_ns)
            return fail(HIPMR_E_INVALID, "arrival times must be non-decreasing");
    }
    std::vector<hipmr_sjob> copy(jobs, jobs + njobs);
    std::vector<char> ok(njobs, 1);
    for (int32_t k = 0; k < njobs; ++k) {
        hipmr_status st = validate_job(s, &copy[k]);
        if (st != HIPMR_OK) {
            // rejected at admission: reported, never packed
            done[k] = hipmr_completion{(1ull << 62) + (uint64_t)k, st, 0, 0, 0, 0};
            ok[k] = 0;
            copy[k].n = 0;
            copy[k].tmpl = -1;
        } else {
            ++valid;
        }
    }
    std::vector<hipmr_sjob> sched;
    std::vector<int32_t> index;
    for (int32_t k = 0; k < njobs; ++k)
        if (ok[k]) {
            sched.push_back(copy[k]);
            index.push_back(k);
        }
    std::vector<hipmr_completion> out(sched.size());
    {
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->sched) return fail(HIPMR_E_INVALID, "a schedule is already running on this server");
        s->sched = sched.data();
        s->sched_n = (int32_t)sched.size();
        s->sched_next = 0;
        s->sched_done = 0;
        s->sched_out = out.data();
        s->unfinished += (int64_t)sched.size();
        s->sched_t0 = now_ns();
    }
    s->cv_work.notify_one();
    {
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.wait(lk, [&] { return s->sched_done == s->sched_n; });
        s->sched = nullptr;
        s->sched_out = nullptr;
    }
    for (size_t k = 0; k < sched.size(); ++k) {
        done[index[k]] = out[k];
        done[index[k]].ticket = (uint64_t)index[k];
        done[index[k]].arrival_ns -= s->sched_t0;
        done[index[k]].launch_ns -= s->sched_t0;
        done[index[k]].done_ns -= s->sched_t0;
    }
    for (int32_t k = 0; k < njobs; ++k)
        if (!ok[k]) done[k].ticket = (uint64_t)k;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->worker_status != HIPMR_OK) return fail(s->worker_status, s->worker_error);
    return HIPMR_OK;
}

void hipmr_server_destroy(hipmr_server_t s) {
    if (!s) return;
    s->stop = true;
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    delete s;   // the destructor frees the streams, pinned buffers and module
}

}  // extern "C"
