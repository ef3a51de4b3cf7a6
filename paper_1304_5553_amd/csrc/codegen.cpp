// Code generation: HIP device templates for gfx950 and their rendering.
//
// The paper generates device code at run time by textual keyword replacement,
// optionally combined with preprocessor macros, and by templating when
// control flow is needed (section "Generating Code"); run-time specialisation
// bakes constants, types and trip counts into the source (section "The Cost
// of Flexibility"), and the user's expression lands inside the inner loop
// with no function-pointer indirection (section "High-Performance
// Abstractions").  Here the templates below carry @@KEY@@ markers that are
// replaced by the signature's types, the user's statement / map / reduce /
// neutral text and the launch constants (block size, vector chunks per
// thread, elements per chunk, index width).
//
// Kernel family (all wave64, no atomics, no LDS beyond the reduction tree):
//   ew_vec   grid-stride over VEC-element chunks; each thread keeps IPT chunks
//            of every accessed array in flight (16-byte loads/stores), runs the
//            statement per element from registers, stores back;
//   ew_sca   one element per step (any access pattern);
//   rs1_vec  same loads; per-thread accumulators (one per in-flight chunk),
//            folded pairwise, then a wave64 butterfly (cross-lane shuffles)
//            and an LDS tree across the block's waves -> one partial per block;
//   rs1_sca  one element per step, same tree;
//   rs2      one block folds the G partials in a fixed order -> *out.
#include <cstdio>
#include <sstream>

#include "common.h"
#include "internal.h"

namespace hipmr {
namespace {

const char* kPrelude = R"HIP(
// ---- hipmr device prelude (gfx950) ----
#ifndef INFINITY
#define INFINITY __builtin_huge_valf()
#endif
#ifndef NAN
#define NAN __builtin_nanf("")
#endif
#ifndef HUGE_VALF
#define HUGE_VALF __builtin_huge_valf()
#endif
#ifndef HUGE_VAL
#define HUGE_VAL __builtin_huge_val()
#endif
#ifndef FLT_MAX
#define FLT_MAX 3.40282347e+38F
#endif
#ifndef FLT_MIN
#define FLT_MIN 1.17549435e-38F
#endif
#ifndef DBL_MAX
#define DBL_MAX 1.7976931348623157e+308
#endif
#ifndef INT_MAX
#define INT_MAX 2147483647
#endif
#ifndef INT_MIN
#define INT_MIN (-2147483647 - 1)
#endif
#ifndef UINT_MAX
#define UINT_MAX 4294967295U
#endif
#ifndef LLONG_MAX
#define LLONG_MAX 9223372036854775807LL
#endif
#ifndef LLONG_MIN
#define LLONG_MIN (-9223372036854775807LL - 1LL)
#endif

typedef unsigned int hipmr_u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int hipmr_u32x2 __attribute__((ext_vector_type(2)));

// Storage-only number formats: a read converts exactly to float, arithmetic
// happens in float, a store rounds to nearest even.
struct hipmr_bf16 {
  unsigned short bits;
  __device__ __forceinline__ operator float() const {
    return __uint_as_float((unsigned int)bits << 16);
  }
  __device__ __forceinline__ hipmr_bf16& operator=(float f) {
    unsigned int u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) {
      bits = (unsigned short)((u >> 16) | 0x40u);          // quiet NaN
    } else {
      u += 0x7fffu + ((u >> 16) & 1u);                      // round to nearest even
      bits = (unsigned short)(u >> 16);
    }
    return *this;
  }
  __device__ __forceinline__ hipmr_bf16& operator+=(float f) { return *this = (float)*this + f; }
  __device__ __forceinline__ hipmr_bf16& operator-=(float f) { return *this = (float)*this - f; }
  __device__ __forceinline__ hipmr_bf16& operator*=(float f) { return *this = (float)*this * f; }
  __device__ __forceinline__ hipmr_bf16& operator/=(float f) { return *this = (float)*this / f; }
};

struct hipmr_f16 {
  _Float16 h;
  __device__ __forceinline__ operator float() const { return (float)h; }
  __device__ __forceinline__ hipmr_f16& operator=(float f) { h = (_Float16)f; return *this; }
  __device__ __forceinline__ hipmr_f16& operator+=(float f) { return *this = (float)*this + f; }
  __device__ __forceinline__ hipmr_f16& operator-=(float f) { return *this = (float)*this - f; }
  __device__ __forceinline__ hipmr_f16& operator*=(float f) { return *this = (float)*this * f; }
  __device__ __forceinline__ hipmr_f16& operator/=(float f) { return *this = (float)*this / f; }
};

// OCP FP8 E4M3 ("fn"): gfx950's conversion instructions use the OCP encoding.
struct hipmr_fp8 {
  unsigned char bits;
  __device__ __forceinline__ operator float() const {
    return __builtin_amdgcn_cvt_f32_fp8((int)bits, 0);
  }
  __device__ __forceinline__ hipmr_fp8& operator=(float f) {
    const float c = (f != f) ? f : __builtin_fminf(__builtin_fmaxf(f, -448.0f), 448.0f);
    bits = (unsigned char)(__builtin_amdgcn_cvt_pk_fp8_f32(c, c, 0, false) & 0xff);
    return *this;
  }
  __device__ __forceinline__ hipmr_fp8& operator+=(float f) { return *this = (float)*this + f; }
  __device__ __forceinline__ hipmr_fp8& operator-=(float f) { return *this = (float)*this - f; }
  __device__ __forceinline__ hipmr_fp8& operator*=(float f) { return *this = (float)*this * f; }
  __device__ __forceinline__ hipmr_fp8& operator/=(float f) { return *this = (float)*this / f; }
};

// Complex values with float components (real, imaginary).
struct hipmr_c64 {
  float re, im;
  hipmr_c64() = default;
  __device__ __forceinline__ constexpr hipmr_c64(float r, float i) : re(r), im(i) {}
  __device__ __forceinline__ constexpr hipmr_c64(float r) : re(r), im(0.0f) {}
  __device__ __forceinline__ constexpr hipmr_c64(double r) : re((float)r), im(0.0f) {}
  __device__ __forceinline__ constexpr hipmr_c64(int r) : re((float)r), im(0.0f) {}
  __device__ __forceinline__ constexpr hipmr_c64(unsigned int r) : re((float)r), im(0.0f) {}
  __device__ __forceinline__ constexpr hipmr_c64(long long r) : re((float)r), im(0.0f) {}
  __device__ __forceinline__ hipmr_c64& operator+=(hipmr_c64 b) { re += b.re; im += b.im; return *this; }
  __device__ __forceinline__ hipmr_c64& operator-=(hipmr_c64 b) { re -= b.re; im -= b.im; return *this; }
  __device__ __forceinline__ hipmr_c64& operator*=(hipmr_c64 b) {
    const float r = re * b.re - im * b.im;
    im = re * b.im + im * b.re;
    re = r;
    return *this;
  }
};
__device__ __forceinline__ hipmr_c64 operator+(hipmr_c64 a, hipmr_c64 b) { return hipmr_c64(a.re + b.re, a.im + b.im); }
__device__ __forceinline__ hipmr_c64 operator-(hipmr_c64 a, hipmr_c64 b) { return hipmr_c64(a.re - b.re, a.im - b.im); }
__device__ __forceinline__ hipmr_c64 operator-(hipmr_c64 a) { return hipmr_c64(-a.re, -a.im); }
__device__ __forceinline__ hipmr_c64 operator+(hipmr_c64 a) { return a; }
__device__ __forceinline__ hipmr_c64 operator*(hipmr_c64 a, hipmr_c64 b) {
  return hipmr_c64(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
__device__ __forceinline__ hipmr_c64 conj(hipmr_c64 z) { return hipmr_c64(z.re, -z.im); }
__device__ __forceinline__ float real(hipmr_c64 z) { return z.re; }
__device__ __forceinline__ float imag(hipmr_c64 z) { return z.im; }
__device__ __forceinline__ float abs(hipmr_c64 z) { return __builtin_sqrtf(z.re * z.re + z.im * z.im); }
__device__ __forceinline__ hipmr_c64 __shfl_xor(hipmr_c64 v, int m, int w) {
  return hipmr_c64(__shfl_xor(v.re, m, w), __shfl_xor(v.im, m, w));
}
__device__ __forceinline__ hipmr_c64 __shfl_up(hipmr_c64 v, unsigned int d, int w) {
  return hipmr_c64(__shfl_up(v.re, d, w), __shfl_up(v.im, d, w));
}
__device__ __forceinline__ hipmr_c64 __shfl(hipmr_c64 v, int l, int w) {
  return hipmr_c64(__shfl(v.re, l, w), __shfl(v.im, l, w));
}

// A vector chunk of N elements held in registers.
template <typename T, int N> struct hipmr_pack { T v[N]; };

template <int B> struct hipmr_word;
template <> struct hipmr_word<1> { typedef unsigned char t; };
template <> struct hipmr_word<2> { typedef unsigned short t; };
template <> struct hipmr_word<4> { typedef unsigned int t; };
template <> struct hipmr_word<8> { typedef hipmr_u32x2 t; };
template <> struct hipmr_word<16> { typedef hipmr_u32x4 t; };

// Loads / stores one chunk with the widest (<= 16-byte) accesses its size
// allows; NT selects streaming (non-temporal) accesses.
template <bool NT, typename T, int N>
__device__ __forceinline__ void hipmr_load(hipmr_pack<T, N>& p, const T* src) {
  constexpr int B = (int)sizeof(T) * N;
  constexpr int W = B >= 16 ? 16 : B;
  typedef typename hipmr_word<W>::t word;
  word tmp[B / W];
  const word* s = reinterpret_cast<const word*>(src);
#pragma unroll
  for (int k = 0; k < B / W; ++k) {
    if constexpr (NT) tmp[k] = __builtin_nontemporal_load(s + k);
    else tmp[k] = s[k];
  }
  __builtin_memcpy(&p, tmp, B);
}

// A read-only chunk of N FP8 values kept as 32-bit words: elements 2k and
// 2k + 1 decode together with the packed conversion instruction (one
// instruction per pair; the pair's two reads share it), no byte extraction.
typedef float hipmr_f32x2 __attribute__((ext_vector_type(2)));
template <int N> struct hipmr_fp8_words {
  unsigned int w[N / 4];
  __device__ __forceinline__ float operator[](int j) const {
    const int word = (int)w[j >> 2];
    const hipmr_f32x2 pair = (j & 2) ? __builtin_amdgcn_cvt_pk_f32_fp8(word, true)
                                     : __builtin_amdgcn_cvt_pk_f32_fp8(word, false);
    return (j & 1) ? pair.y : pair.x;
  }
};
template <int N> struct hipmr_pack_fp8ro { hipmr_fp8_words<N> v; };

template <bool NT, int N>
__device__ __forceinline__ void hipmr_load(hipmr_pack_fp8ro<N>& p, const hipmr_fp8* src) {
  hipmr_pack<hipmr_fp8, N> raw;
  hipmr_load<NT>(raw, src);
  __builtin_memcpy(&p, &raw, N);
}

// A chunk wider than 16 bytes leaves in several store instructions, each
// covering every other 16 bytes of the lanes' lines: streaming stores would
// write those half lines out unmerged, so wide chunks are stored temporally
// (the L2 merges them).
template <bool NT, typename T, int N>
__device__ __forceinline__ void hipmr_store(T* dst, const hipmr_pack<T, N>& p) {
  constexpr int B = (int)sizeof(T) * N;
  constexpr int W = B >= 16 ? 16 : B;
  typedef typename hipmr_word<W>::t word;
  word tmp[B / W];
  __builtin_memcpy(tmp, &p, B);
  word* d = reinterpret_cast<word*>(dst);
#pragma unroll
  for (int k = 0; k < B / W; ++k) {
    if constexpr (NT && B <= 16) __builtin_nontemporal_store(tmp[k], d + k);
    else d[k] = tmp[k];
  }
}
)HIP";

// Reduction helpers; rendered after hipmr_acc and hipmr_combine are defined.
const char* kReduceHelpers = R"HIP(
// wave64 butterfly then an LDS tree over the block's waves; the result is
// valid in thread 0.  The order of combination is fixed by the block size.
template <int B>
__device__ __forceinline__ hipmr_acc hipmr_block_reduce(hipmr_acc v, hipmr_acc neutral) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = hipmr_combine(v, __shfl_xor(v, m, 64));
  if constexpr (B > 64) {
    // W waves (any count up to 16): lanes >= W of wave 0 hold the neutral
    // element and the butterfly spans the next power of two >= W
    constexpr int W = B / 64;
    constexpr int P = W <= 2 ? 2 : W <= 4 ? 4 : W <= 8 ? 8 : 16;
    __shared__ hipmr_acc hipmr_lds[W];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) hipmr_lds[w] = v;
    __syncthreads();
    if (w == 0) {
      v = l < W ? hipmr_lds[l] : neutral;
#pragma unroll
      for (int m = P / 2; m >= 1; m >>= 1) v = hipmr_combine(v, __shfl_xor(v, m, 64));
    }
  }
  return v;
}

// pairwise fold of a thread's U accumulators into a[0]
template <int U>
__device__ __forceinline__ hipmr_acc hipmr_fold(hipmr_acc* a) {
#pragma unroll
  for (int s = 1; s < U; s *= 2) {
#pragma unroll
    for (int u = 0; u + s < U; u += 2 * s) a[u] = hipmr_combine(a[u], a[u + s]);
  }
  return a[0];
}
)HIP";

const char* kEwVector = R"HIP(
extern "C" __global__ void __launch_bounds__(@@BLOCK@@)
@@KNAME@@(@@PARAMS@@, long long hipmr_n, long long hipmr_head)
{
  typedef @@IDX@@ hipmr_idx;
  constexpr int HIPMR_B = @@BLOCK@@, HIPMR_U = @@IPT@@, HIPMR_V = @@VEC@@;
  constexpr bool HIPMR_NTL = @@NTL@@, HIPMR_NTS = @@NTS@@;
  const hipmr_idx n = (hipmr_idx)hipmr_n;
  // elements [0, head) precede the first aligned chunk; [t0, n) is the ragged tail
  const long long hipmr_h = hipmr_head < hipmr_n ? hipmr_head : hipmr_n;
  const long long hipmr_nc = (hipmr_n - hipmr_h) / HIPMR_V;
  const long long hipmr_t0 = hipmr_h + hipmr_nc * HIPMR_V;
  if (blockIdx.x == 0) {
    if ((long long)threadIdx.x < hipmr_h) {
      const hipmr_idx i = (hipmr_idx)threadIdx.x;
      { @@STMT@@; }
    }
    if ((long long)threadIdx.x < hipmr_n - hipmr_t0) {
      const hipmr_idx i = (hipmr_idx)(hipmr_t0 + threadIdx.x);
      { @@STMT@@; }
    }
  }
  const long long hipmr_step = (long long)gridDim.x * (HIPMR_B * HIPMR_U);
  long long hipmr_c0 = (long long)blockIdx.x * (HIPMR_B * HIPMR_U) + threadIdx.x;
  for (; hipmr_c0 + (HIPMR_U - 1) * HIPMR_B < hipmr_nc; hipmr_c0 += hipmr_step) {
    @@DECL_PACKS@@
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < HIPMR_U; ++hipmr_u) {
      const long long hipmr_off = hipmr_h + (hipmr_c0 + hipmr_u * HIPMR_B) * HIPMR_V;
      @@LOADS@@
    }
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < HIPMR_U; ++hipmr_u) {
      const long long hipmr_off = hipmr_h + (hipmr_c0 + hipmr_u * HIPMR_B) * HIPMR_V;
#pragma unroll
      for (int hipmr_j = 0; hipmr_j < HIPMR_V; ++hipmr_j) {
        const hipmr_idx i = (hipmr_idx)(hipmr_off + hipmr_j);
        { @@VSTMT@@; }
      }
      @@STORES@@
    }
  }
  if (hipmr_c0 < hipmr_nc) {
    @@DECL_PACKS@@
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < HIPMR_U; ++hipmr_u) {
      const long long hipmr_c = hipmr_c0 + hipmr_u * HIPMR_B;
      if (hipmr_c < hipmr_nc) {
        const long long hipmr_off = hipmr_h + hipmr_c * HIPMR_V;
        @@LOADS@@
      }
    }
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < HIPMR_U; ++hipmr_u) {
      const long long hipmr_c = hipmr_c0 + hipmr_u * HIPMR_B;
      if (hipmr_c < hipmr_nc) {
        const long long hipmr_off = hipmr_h + hipmr_c * HIPMR_V;
#pragma unroll
        for (int hipmr_j = 0; hipmr_j < HIPMR_V; ++hipmr_j) {
          const hipmr_idx i = (hipmr_idx)(hipmr_off + hipmr_j);
          { @@VSTMT@@; }
        }
        @@STORES@@
      }
    }
  }
}
)HIP";

// The vector elementwise kernel for statements with shifted reads
// name[i + E]: per chunk, each distinct shifted read is one unaligned load of
// V elements from name + off + E.  A chunk whose shifted loads would leave
// [0, n) (within |E| of either end) runs the statement one element at a time
// instead, with the statement's own guards.
const char* kShiftHelpers = R"HIP(
// 16 bytes at 4-byte alignment: one dwordx4 load (the memory system accepts
// dword-aligned multi-dword accesses); narrower element types go by memcpy
typedef unsigned int hipmr_u32x4u __attribute__((ext_vector_type(4), aligned(4)));

template <typename T, int N>
__device__ __forceinline__ void hipmr_loadu(hipmr_pack<T, N>& p, const T* src) {
  if constexpr (sizeof(p) % 16 == 0 && alignof(T) >= 4) {
    hipmr_u32x4u w[sizeof(p) / 16];
#pragma unroll
    for (int k = 0; k < (int)(sizeof(p) / 16); ++k) w[k] = reinterpret_cast<const hipmr_u32x4u*>(src)[k];
    __builtin_memcpy(&p, w, sizeof(p));
  } else {
    __builtin_memcpy(&p, src, sizeof(p));
  }
}

// XCD-aware order: workgroups go round-robin to the 8 XCDs, each with its own
// L2.  Renumbered, each XCD takes a contiguous run of chunks, so the
// neighbouring elements a shifted read reaches were loaded by the same XCD.
// the window start off + s clamped into [0, hi] (hi = n - V >= 0, 0 <= off <= hi),
// without forming off + s when it would leave that range (s may be huge)
__device__ __forceinline__ long long hipmr_clampv(long long off, long long s, long long hi) {
  return s < -off ? 0 : (s > hi - off ? hi : off + s);
}

__device__ __forceinline__ unsigned hipmr_xcd_block() {
  const unsigned x = blockIdx.x % 8u, q = gridDim.x / 8u, r = gridDim.x % 8u;
  return x * q + (x < r ? x : r) + blockIdx.x / 8u;
}
)HIP";

const char* kEwVectorShift = R"HIP(
extern "C" __global__ void __launch_bounds__(@@BLOCK@@)
@@KNAME@@(@@PARAMS@@, long long hipmr_n, long long hipmr_head)
{
  typedef @@IDX@@ hipmr_idx;
  constexpr int HIPMR_B = @@BLOCK@@, HIPMR_U = @@IPT@@, HIPMR_V = @@VEC@@;
  constexpr bool HIPMR_NTL = @@NTL@@, HIPMR_NTS = @@NTS@@;
  const hipmr_idx n = (hipmr_idx)hipmr_n;
  @@SHIFT_INIT@@
  const long long hipmr_h = hipmr_head < hipmr_n ? hipmr_head : hipmr_n;
  const long long hipmr_nc = (hipmr_n - hipmr_h) / HIPMR_V;
  const long long hipmr_t0 = hipmr_h + hipmr_nc * HIPMR_V;
  if (blockIdx.x == 0) {
    if ((long long)threadIdx.x < hipmr_h) {
      const hipmr_idx i = (hipmr_idx)threadIdx.x;
      { @@STMT@@; }
    }
    if ((long long)threadIdx.x < hipmr_n - hipmr_t0) {
      const hipmr_idx i = (hipmr_idx)(hipmr_t0 + threadIdx.x);
      { @@STMT@@; }
    }
  }
  const long long hipmr_step = (long long)gridDim.x * (HIPMR_B * HIPMR_U);
  for (long long hipmr_c0 = (long long)hipmr_xcd_block() * (HIPMR_B * HIPMR_U) + threadIdx.x;
       hipmr_c0 < hipmr_nc; hipmr_c0 += hipmr_step) {
    @@DECL_PACKS@@
    @@SHIFT_PACKS@@
    bool hipmr_vec[HIPMR_U];
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < HIPMR_U; ++hipmr_u) {
      const long long hipmr_c = hipmr_c0 + hipmr_u * HIPMR_B;
      const long long hipmr_off = hipmr_h + hipmr_c * HIPMR_V;
      hipmr_vec[hipmr_u] = hipmr_c < hipmr_nc && hipmr_smin >= -hipmr_off &&
                           hipmr_smax <= hipmr_n - HIPMR_V - hipmr_off;   // no overflow for any distance
      if (hipmr_vec[hipmr_u]) {
        @@LOADS@@
        @@SHIFT_LOADS@@
      }
    }
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < HIPMR_U; ++hipmr_u) {
      const long long hipmr_c = hipmr_c0 + hipmr_u * HIPMR_B;
      const long long hipmr_off = hipmr_h + hipmr_c * HIPMR_V;
      if (hipmr_vec[hipmr_u]) {
#pragma unroll
        for (int hipmr_j = 0; hipmr_j < HIPMR_V; ++hipmr_j) {
          const hipmr_idx i = (hipmr_idx)(hipmr_off + hipmr_j);
          { @@VSTMT@@; }
        }
        @@STORES@@
      } else if (hipmr_c < hipmr_nc) {
        for (int hipmr_j = 0; hipmr_j < HIPMR_V; ++hipmr_j) {
          const hipmr_idx i = (hipmr_idx)(hipmr_off + hipmr_j);
          { @@STMT@@; }
        }
      }
    }
  }
}
)HIP";

const char* kEwScalar = R"HIP(
extern "C" __global__ void __launch_bounds__(@@BLOCK@@)
@@KNAME@@(@@PARAMS@@, long long hipmr_n, long long hipmr_head)
{
  typedef @@IDX@@ hipmr_idx;
  const hipmr_idx n = (hipmr_idx)hipmr_n;
  const long long hipmr_step = (long long)gridDim.x * @@BLOCK@@;
#pragma unroll @@IPT@@
  for (long long hipmr_k = (long long)blockIdx.x * @@BLOCK@@ + threadIdx.x; hipmr_k < hipmr_n;
       hipmr_k += hipmr_step) {
    const hipmr_idx i = (hipmr_idx)hipmr_k;
    { @@STMT@@; }
  }
}
)HIP";

const char* kRedS1Vector = R"HIP(
extern "C" __global__ void __launch_bounds__(@@BLOCK@@)
@@KNAME@@(@@PARAMS@@, long long hipmr_n, long long hipmr_head,
          hipmr_acc* __restrict__ hipmr_partial)
{
  typedef @@IDX@@ hipmr_idx;
  constexpr int HIPMR_B = @@BLOCK@@, HIPMR_U = @@IPT@@, HIPMR_V = @@VEC@@;
  constexpr bool HIPMR_NTL = @@NTL@@, HIPMR_NTS = @@NTS@@;
  const hipmr_idx n = (hipmr_idx)hipmr_n;
  const hipmr_acc hipmr_neutral = (hipmr_acc)(@@NEUTRAL@@);
  hipmr_acc hipmr_a[HIPMR_U];
#pragma unroll
  for (int u = 0; u < HIPMR_U; ++u) hipmr_a[u] = hipmr_neutral;
  const long long hipmr_h = hipmr_head < hipmr_n ? hipmr_head : hipmr_n;
  const long long hipmr_nc = (hipmr_n - hipmr_h) / HIPMR_V;
  const long long hipmr_t0 = hipmr_h + hipmr_nc * HIPMR_V;
  if (blockIdx.x == 0) {
    if ((long long)threadIdx.x < hipmr_h) {
      const hipmr_idx i = (hipmr_idx)threadIdx.x;
      hipmr_a[0] = hipmr_combine(hipmr_a[0], (hipmr_acc)(@@MAP@@));
    }
    if ((long long)threadIdx.x < hipmr_n - hipmr_t0) {
      const hipmr_idx i = (hipmr_idx)(hipmr_t0 + threadIdx.x);
      hipmr_a[0] = hipmr_combine(hipmr_a[0], (hipmr_acc)(@@MAP@@));
    }
  }
  const long long hipmr_step = (long long)gridDim.x * (HIPMR_B * HIPMR_U);
  long long hipmr_c0 = (long long)blockIdx.x * (HIPMR_B * HIPMR_U) + threadIdx.x;
  for (; hipmr_c0 + (HIPMR_U - 1) * HIPMR_B < hipmr_nc; hipmr_c0 += hipmr_step) {
    @@DECL_PACKS@@
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < HIPMR_U; ++hipmr_u) {
      const long long hipmr_off = hipmr_h + (hipmr_c0 + hipmr_u * HIPMR_B) * HIPMR_V;
      @@LOADS@@
    }
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < HIPMR_U; ++hipmr_u) {
      const long long hipmr_off = hipmr_h + (hipmr_c0 + hipmr_u * HIPMR_B) * HIPMR_V;
#pragma unroll
      for (int hipmr_j = 0; hipmr_j < HIPMR_V; ++hipmr_j) {
        const hipmr_idx i = (hipmr_idx)(hipmr_off + hipmr_j);
        hipmr_a[hipmr_u] = hipmr_combine(hipmr_a[hipmr_u], (hipmr_acc)(@@VMAP@@));
      }
    }
  }
  if (hipmr_c0 < hipmr_nc) {
    @@DECL_PACKS@@
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < HIPMR_U; ++hipmr_u) {
      const long long hipmr_c = hipmr_c0 + hipmr_u * HIPMR_B;
      if (hipmr_c < hipmr_nc) {
        const long long hipmr_off = hipmr_h + hipmr_c * HIPMR_V;
        @@LOADS@@
      }
    }
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < HIPMR_U; ++hipmr_u) {
      const long long hipmr_c = hipmr_c0 + hipmr_u * HIPMR_B;
      if (hipmr_c < hipmr_nc) {
        const long long hipmr_off = hipmr_h + hipmr_c * HIPMR_V;
#pragma unroll
        for (int hipmr_j = 0; hipmr_j < HIPMR_V; ++hipmr_j) {
          const hipmr_idx i = (hipmr_idx)(hipmr_off + hipmr_j);
          hipmr_a[hipmr_u] = hipmr_combine(hipmr_a[hipmr_u], (hipmr_acc)(@@VMAP@@));
        }
      }
    }
  }
  hipmr_acc hipmr_r = hipmr_fold<HIPMR_U>(hipmr_a);
  hipmr_r = hipmr_block_reduce<HIPMR_B>(hipmr_r, hipmr_neutral);
  if (threadIdx.x == 0) hipmr_partial[blockIdx.x] = hipmr_r;
}
)HIP";

const char* kRedS1Scalar = R"HIP(
extern "C" __global__ void __launch_bounds__(@@BLOCK@@)
@@KNAME@@(@@PARAMS@@, long long hipmr_n, long long hipmr_head,
          hipmr_acc* __restrict__ hipmr_partial)
{
  typedef @@IDX@@ hipmr_idx;
  const hipmr_idx n = (hipmr_idx)hipmr_n;
  const hipmr_acc hipmr_neutral = (hipmr_acc)(@@NEUTRAL@@);
  hipmr_acc hipmr_r = hipmr_neutral;
  const long long hipmr_step = (long long)gridDim.x * @@BLOCK@@;
#pragma unroll @@IPT@@
  for (long long hipmr_k = (long long)blockIdx.x * @@BLOCK@@ + threadIdx.x; hipmr_k < hipmr_n;
       hipmr_k += hipmr_step) {
    const hipmr_idx i = (hipmr_idx)hipmr_k;
    hipmr_r = hipmr_combine(hipmr_r, (hipmr_acc)(@@MAP@@));
  }
  hipmr_r = hipmr_block_reduce<@@BLOCK@@>(hipmr_r, hipmr_neutral);
  if (threadIdx.x == 0) hipmr_partial[blockIdx.x] = hipmr_r;
}
)HIP";

// Reduce stage 1 for maps with shifted reads: as kEwVectorShift, each
// distinct shifted read is one unaligned chunk load, chunks within the largest
// distance of either end are mapped one element at a time, and workgroups
// take XCD-contiguous runs of chunks.  Each lane folds its chunks in order
// into U accumulators; the partial of workgroup b lands in partial[b].
const char* kRedS1VectorShift = R"HIP(
extern "C" __global__ void __launch_bounds__(@@BLOCK@@)
@@KNAME@@(@@PARAMS@@, long long hipmr_n, long long hipmr_head,
          hipmr_acc* __restrict__ hipmr_partial)
{
  typedef @@IDX@@ hipmr_idx;
  constexpr int HIPMR_B = @@BLOCK@@, HIPMR_U = @@IPT@@, HIPMR_V = @@VEC@@;
  constexpr bool HIPMR_NTL = @@NTL@@, HIPMR_NTS = @@NTS@@;
  const hipmr_idx n = (hipmr_idx)hipmr_n;
  @@SHIFT_INIT@@
  const hipmr_acc hipmr_neutral = (hipmr_acc)(@@NEUTRAL@@);
  hipmr_acc hipmr_a[HIPMR_U];
#pragma unroll
  for (int u = 0; u < HIPMR_U; ++u) hipmr_a[u] = hipmr_neutral;
  const long long hipmr_h = hipmr_head < hipmr_n ? hipmr_head : hipmr_n;
  const long long hipmr_nc = (hipmr_n - hipmr_h) / HIPMR_V;
  const long long hipmr_t0 = hipmr_h + hipmr_nc * HIPMR_V;
  if (blockIdx.x == 0) {
    if ((long long)threadIdx.x < hipmr_h) {
      const hipmr_idx i = (hipmr_idx)threadIdx.x;
      hipmr_a[0] = hipmr_combine(hipmr_a[0], (hipmr_acc)(@@MAP@@));
    }
    if ((long long)threadIdx.x < hipmr_n - hipmr_t0) {
      const hipmr_idx i = (hipmr_idx)(hipmr_t0 + threadIdx.x);
      hipmr_a[0] = hipmr_combine(hipmr_a[0], (hipmr_acc)(@@MAP@@));
    }
  }
  const long long hipmr_step = (long long)gridDim.x * (HIPMR_B * HIPMR_U);
  for (long long hipmr_c0 = (long long)hipmr_xcd_block() * (HIPMR_B * HIPMR_U) + threadIdx.x;
       hipmr_c0 < hipmr_nc; hipmr_c0 += hipmr_step) {
    @@DECL_PACKS@@
    @@SHIFT_PACKS@@
    bool hipmr_vec[HIPMR_U];
    // every lane loads every chunk, from a clamped in-range window where its
    // chunk is past the end or within a shifted read's distance of an end
    // (those chunks are then evaluated element by element): no branch
    // separates the loads, so they all stay in flight together
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < HIPMR_U; ++hipmr_u) {
      const long long hipmr_c = hipmr_c0 + hipmr_u * HIPMR_B;
      const long long hipmr_off = hipmr_c < hipmr_nc ? hipmr_h + hipmr_c * HIPMR_V : hipmr_h;
      hipmr_vec[hipmr_u] = hipmr_c < hipmr_nc && hipmr_smin >= -hipmr_off &&
                           hipmr_smax <= hipmr_n - HIPMR_V - hipmr_off;   // no overflow for any distance
      @@LOADS@@
      @@SHIFT_LOADS@@
    }
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < HIPMR_U; ++hipmr_u) {
      const long long hipmr_c = hipmr_c0 + hipmr_u * HIPMR_B;
      const long long hipmr_off = hipmr_h + hipmr_c * HIPMR_V;
      if (hipmr_vec[hipmr_u]) {
#pragma unroll
        for (int hipmr_j = 0; hipmr_j < HIPMR_V; ++hipmr_j) {
          const hipmr_idx i = (hipmr_idx)(hipmr_off + hipmr_j);
          hipmr_a[hipmr_u] = hipmr_combine(hipmr_a[hipmr_u], (hipmr_acc)(@@VMAP@@));
        }
      } else if (hipmr_c < hipmr_nc) {
        for (int hipmr_j = 0; hipmr_j < HIPMR_V; ++hipmr_j) {
          const hipmr_idx i = (hipmr_idx)(hipmr_off + hipmr_j);
          hipmr_a[hipmr_u] = hipmr_combine(hipmr_a[hipmr_u], (hipmr_acc)(@@MAP@@));
        }
      }
    }
  }
  hipmr_acc hipmr_r = hipmr_fold<HIPMR_U>(hipmr_a);
  hipmr_r = hipmr_block_reduce<HIPMR_B>(hipmr_r, hipmr_neutral);
  if (threadIdx.x == 0) hipmr_partial[blockIdx.x] = hipmr_r;
}
)HIP";

const char* kRedS2 = R"HIP(
extern "C" __global__ void __launch_bounds__(@@BLOCK@@)
@@KNAME@@(const hipmr_acc* __restrict__ hipmr_partial, int hipmr_g,
          hipmr_acc* __restrict__ hipmr_out)
{
  const hipmr_acc hipmr_neutral = (hipmr_acc)(@@NEUTRAL@@);
  hipmr_acc hipmr_r = hipmr_neutral;
  for (int k = threadIdx.x; k < hipmr_g; k += @@BLOCK@@)
    hipmr_r = hipmr_combine(hipmr_r, hipmr_partial[k]);
  hipmr_r = hipmr_block_reduce<@@BLOCK@@>(hipmr_r, hipmr_neutral);
  if (threadIdx.x == 0) *hipmr_out = hipmr_r;
}
)HIP";


// Compensated FP32 accumulation (precision extension).  Error-free
// transformations must not be contracted into FMAs.
const char* kCompHelpers = R"HIP(
#pragma clang fp contract(off)
// (hi, lo): an unevaluated sum of two floats
struct hipmr_ff { float hi, lo; };
struct hipmr_dd { double hi, lo; };

// Kahan: s + (-c) carries the running sum; c holds the rounding lost so far.
// Once the sum is infinite (or NaN) the correction is dropped, so that an
// infinity is not turned into a NaN by inf - inf.
__device__ __forceinline__ void hipmr_kahan_add(float& s, float& c, float v) {
  const float y = v - c;
  const float t = s + y;
  c = __builtin_isfinite(t) ? (t - s) - y : 0.0f;
  s = t;
}

// Knuth's TwoSum: a + b = s + e exactly, no ordering assumption
__device__ __forceinline__ hipmr_ff hipmr_two_sum(float a, float b) {
  const float s = a + b;
  const float bb = s - a;
  return {s, __builtin_isfinite(s) ? (a - (s - bb)) + (b - bb) : 0.0f};
}
__device__ __forceinline__ hipmr_ff hipmr_ff_add(hipmr_ff x, hipmr_ff y) {
  const hipmr_ff s = hipmr_two_sum(x.hi, y.hi);
  return hipmr_two_sum(s.hi, s.lo + (x.lo + y.lo));
}
__device__ __forceinline__ hipmr_dd hipmr_two_sum_d(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  return {s, __builtin_isfinite(s) ? (a - (s - bb)) + (b - bb) : 0.0};
}
__device__ __forceinline__ hipmr_dd hipmr_dd_add(hipmr_dd x, hipmr_dd y) {
  const hipmr_dd s = hipmr_two_sum_d(x.hi, y.hi);
  return hipmr_two_sum_d(s.hi, s.lo + (x.lo + y.lo));
}

// The norm's power-of-two scale from its first pass: the max |map| over
// that pass's block partials (one per block of this grid: both passes use
// the same geometry), then s = 2^-e, e the exponent of the max clamped to
// [-126, 126], so the largest scaled magnitude lies in [1, 2).  Every block
// computes it; block 0 also stores it (float, then double) for the final
// fold.
template <int B>
__device__ __forceinline__ float hipmr_norm_scale(const float* __restrict__ amax,
                                                  float* __restrict__ store) {
  __shared__ float hipmr_scale_lds[B / 64];
  float m = 0.0f;
  for (int k = threadIdx.x; k < (int)gridDim.x; k += B) m = __builtin_elementwise_maximum(m, amax[k]);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) m = __builtin_elementwise_maximum(m, __shfl_xor(m, d, 64));
  if ((threadIdx.x & 63) == 0) hipmr_scale_lds[threadIdx.x >> 6] = m;
  __syncthreads();
  m = hipmr_scale_lds[0];
#pragma unroll
  for (int w = 1; w < B / 64; ++w) m = __builtin_elementwise_maximum(m, hipmr_scale_lds[w]);
  float s = 1.0f;
  if (m > 0.0f) {
    int e = (int)((__float_as_uint(m) >> 23) & 0xffu) - 127;
    e = e < -126 ? -126 : (e > 126 ? 126 : e);
    s = __uint_as_float((unsigned int)(127 - e) << 23);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    store[0] = s;
    *(double*)(store + 2) = (double)s;
  }
  return s;
}

// pairwise sum of one chunk's V terms (fixed tree); the chunk sum then
// enters the compensated accumulator
template <int V>
__device__ __forceinline__ float hipmr_chunk_sum(float* t) {
#pragma unroll
  for (int w = 1; w < V; w *= 2) {
#pragma unroll
    for (int j = 0; j + w < V; j += 2 * w) t[j] += t[j + w];
  }
  return t[0];
}

template <bool SQ>
__device__ __forceinline__ float hipmr_term(float v, float scale) {
  if constexpr (SQ) {
    const float w = v * scale;
    return w * w;
  } else {
    return v;
  }
}

// pairwise combination of (hi, lo) pairs across the wave, then the block
template <int B, typename P, typename F>
__device__ __forceinline__ P hipmr_block_reduce_pair(P v, F add) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    P o;
    o.hi = __shfl_xor(v.hi, m, 64);
    o.lo = __shfl_xor(v.lo, m, 64);
    v = add(v, o);
  }
  if constexpr (B > 64) {
    constexpr int W = B / 64;
    constexpr int PW = W <= 2 ? 2 : W <= 4 ? 4 : W <= 8 ? 8 : 16;
    __shared__ P hipmr_lds_pair[W];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) hipmr_lds_pair[w] = v;
    __syncthreads();
    if (w == 0) {
      if (l < W) v = hipmr_lds_pair[l];
      else { v.hi = 0; v.lo = 0; }
#pragma unroll
      for (int m = PW / 2; m >= 1; m >>= 1) {
        P o;
        o.hi = __shfl_xor(v.hi, m, 64);
        o.lo = __shfl_xor(v.lo, m, 64);
        v = add(v, o);
      }
    }
  }
  return v;
}
)HIP";

// Stage 1 of a compensated sum (or of the norm's sum of squares).
const char* kCompS1Vector = R"HIP(
extern "C" __global__ void __launch_bounds__(@@BLOCK@@)
@@KNAME@@(@@PARAMS@@, long long hipmr_n, long long hipmr_head,
          double* __restrict__ hipmr_partial, const float* __restrict__ hipmr_scale_p)
{
  typedef @@IDX@@ hipmr_idx;
  constexpr int HIPMR_B = @@BLOCK@@, HIPMR_U = @@IPT@@, HIPMR_V = @@VEC@@;
  constexpr bool HIPMR_NTL = @@NTL@@, HIPMR_NTS = @@NTS@@;
  constexpr bool HIPMR_SQ = @@SQUARE@@, HIPMR_RUNS = @@RUNS@@, HIPMR_SCALED = @@SCALED@@;
  const hipmr_idx n = (hipmr_idx)hipmr_n;
  float hipmr_sc = 1.0f;
  if constexpr (HIPMR_SCALED)
    hipmr_sc = hipmr_norm_scale<HIPMR_B>(hipmr_scale_p, (float*)((char*)hipmr_scale_p + @@SCALE_GAP@@));
  float hipmr_s[HIPMR_U], hipmr_e[HIPMR_U];
#pragma unroll
  for (int u = 0; u < HIPMR_U; ++u) { hipmr_s[u] = 0.0f; hipmr_e[u] = 0.0f; }
  const long long hipmr_h = hipmr_head < hipmr_n ? hipmr_head : hipmr_n;
  const long long hipmr_nc = (hipmr_n - hipmr_h) / HIPMR_V;
  const long long hipmr_t0 = hipmr_h + hipmr_nc * HIPMR_V;
  if (blockIdx.x == 0) {
    if ((long long)threadIdx.x < hipmr_h) {
      const hipmr_idx i = (hipmr_idx)threadIdx.x;
      hipmr_kahan_add(hipmr_s[0], hipmr_e[0], hipmr_term<HIPMR_SQ>((float)(@@MAP@@), hipmr_sc));
    }
    if ((long long)threadIdx.x < hipmr_n - hipmr_t0) {
      const hipmr_idx i = (hipmr_idx)(hipmr_t0 + threadIdx.x);
      hipmr_kahan_add(hipmr_s[0], hipmr_e[0], hipmr_term<HIPMR_SQ>((float)(@@MAP@@), hipmr_sc));
    }
  }
  const long long hipmr_step = (long long)gridDim.x * (HIPMR_B * HIPMR_U);
  long long hipmr_c0 = (long long)blockIdx.x * (HIPMR_B * HIPMR_U) + threadIdx.x;
  for (; hipmr_c0 + (HIPMR_U - 1) * HIPMR_B < hipmr_nc; hipmr_c0 += hipmr_step) {
    @@DECL_PACKS@@
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < HIPMR_U; ++hipmr_u) {
      const long long hipmr_off = hipmr_h + (hipmr_c0 + hipmr_u * HIPMR_B) * HIPMR_V;
      @@LOADS@@
    }
    if constexpr (HIPMR_RUNS) {
      // every value is k * 2^-9 with |k| <= 229376: a float sum of at most
      // 64 of them is exact, so one compensated step per run suffices
      float hipmr_run = 0.0f;
#pragma unroll
      for (int hipmr_u = 0; hipmr_u < HIPMR_U; ++hipmr_u) {
        const long long hipmr_off = hipmr_h + (hipmr_c0 + hipmr_u * HIPMR_B) * HIPMR_V;
#pragma unroll
        for (int hipmr_j = 0; hipmr_j < HIPMR_V; ++hipmr_j) {
          const hipmr_idx i = (hipmr_idx)(hipmr_off + hipmr_j);
          hipmr_run += (float)(@@VMAP@@);
        }
      }
      hipmr_kahan_add(hipmr_s[0], hipmr_e[0], hipmr_run);
    } else {
#pragma unroll
      for (int hipmr_u = 0; hipmr_u < HIPMR_U; ++hipmr_u) {
        const long long hipmr_off = hipmr_h + (hipmr_c0 + hipmr_u * HIPMR_B) * HIPMR_V;
        float hipmr_t[HIPMR_V];
#pragma unroll
        for (int hipmr_j = 0; hipmr_j < HIPMR_V; ++hipmr_j) {
          const hipmr_idx i = (hipmr_idx)(hipmr_off + hipmr_j);
          hipmr_t[hipmr_j] = hipmr_term<HIPMR_SQ>((float)(@@VMAP@@), hipmr_sc);
        }
        hipmr_kahan_add(hipmr_s[hipmr_u], hipmr_e[hipmr_u], hipmr_chunk_sum<HIPMR_V>(hipmr_t));
      }
    }
  }
  if (hipmr_c0 < hipmr_nc) {
    @@DECL_PACKS@@
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < HIPMR_U; ++hipmr_u) {
      const long long hipmr_c = hipmr_c0 + hipmr_u * HIPMR_B;
      if (hipmr_c < hipmr_nc) {
        const long long hipmr_off = hipmr_h + hipmr_c * HIPMR_V;
        @@LOADS@@
      }
    }
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < HIPMR_U; ++hipmr_u) {
      const long long hipmr_c = hipmr_c0 + hipmr_u * HIPMR_B;
      if (hipmr_c < hipmr_nc) {
        const long long hipmr_off = hipmr_h + hipmr_c * HIPMR_V;
        float hipmr_t[HIPMR_V];
#pragma unroll
        for (int hipmr_j = 0; hipmr_j < HIPMR_V; ++hipmr_j) {
          const hipmr_idx i = (hipmr_idx)(hipmr_off + hipmr_j);
          hipmr_t[hipmr_j] = hipmr_term<HIPMR_SQ>((float)(@@VMAP@@), hipmr_sc);
        }
        hipmr_kahan_add(hipmr_s[hipmr_u], hipmr_e[hipmr_u], hipmr_chunk_sum<HIPMR_V>(hipmr_t));
      }
    }
  }
  hipmr_ff hipmr_r = {hipmr_s[0], -hipmr_e[0]};
#pragma unroll
  for (int u = 1; u < HIPMR_U; ++u) hipmr_r = hipmr_ff_add(hipmr_r, hipmr_ff{hipmr_s[u], -hipmr_e[u]});
  hipmr_r = hipmr_block_reduce_pair<HIPMR_B>(hipmr_r, [](hipmr_ff a, hipmr_ff b) { return hipmr_ff_add(a, b); });
  if (threadIdx.x == 0)
    hipmr_partial[blockIdx.x] = __builtin_isfinite(hipmr_r.hi) ? (double)hipmr_r.hi + (double)hipmr_r.lo
                                                               : (double)hipmr_r.hi;
}
)HIP";

const char* kCompS1Scalar = R"HIP(
extern "C" __global__ void __launch_bounds__(@@BLOCK@@)
@@KNAME@@(@@PARAMS@@, long long hipmr_n, long long hipmr_head,
          double* __restrict__ hipmr_partial, const float* __restrict__ hipmr_scale_p)
{
  typedef @@IDX@@ hipmr_idx;
  constexpr bool HIPMR_SQ = @@SQUARE@@, HIPMR_SCALED = @@SCALED@@;
  const hipmr_idx n = (hipmr_idx)hipmr_n;
  float hipmr_sc = 1.0f;
  if constexpr (HIPMR_SCALED)
    hipmr_sc = hipmr_norm_scale<@@BLOCK@@>(hipmr_scale_p, (float*)((char*)hipmr_scale_p + @@SCALE_GAP@@));
  float hipmr_s = 0.0f, hipmr_cc = 0.0f;
  const long long hipmr_step = (long long)gridDim.x * @@BLOCK@@;
  for (long long hipmr_k = (long long)blockIdx.x * @@BLOCK@@ + threadIdx.x; hipmr_k < hipmr_n;
       hipmr_k += hipmr_step) {
    const hipmr_idx i = (hipmr_idx)hipmr_k;
    hipmr_kahan_add(hipmr_s, hipmr_cc, hipmr_term<HIPMR_SQ>((float)(@@MAP@@), hipmr_sc));
  }
  hipmr_ff hipmr_r = {hipmr_s, -hipmr_cc};
  hipmr_r = hipmr_block_reduce_pair<@@BLOCK@@>(hipmr_r, [](hipmr_ff a, hipmr_ff b) { return hipmr_ff_add(a, b); });
  if (threadIdx.x == 0)
    hipmr_partial[blockIdx.x] = __builtin_isfinite(hipmr_r.hi) ? (double)hipmr_r.hi + (double)hipmr_r.lo
                                                               : (double)hipmr_r.hi;
}
)HIP";

// Final fold of the FP64 block partials (Neumaier per thread, double-double
// tree), times the per-tensor post scale; the norm finishes as sqrt / scale.
const char* kCompS2 = R"HIP(
extern "C" __global__ void __launch_bounds__(@@BLOCK@@)
@@KNAME@@(const double* __restrict__ hipmr_partial, int hipmr_g, double hipmr_post,
          const double* __restrict__ hipmr_scale64, double* __restrict__ hipmr_out)
{
  constexpr bool NORM = @@NORM@@, SCALED = @@SCALED@@;
  double s = 0.0, c = 0.0;
  for (int k = threadIdx.x; k < hipmr_g; k += @@BLOCK@@) {
    const double v = hipmr_partial[k];
    const double t = s + v;
    if (__builtin_isfinite(t)) c += fabs(s) >= fabs(v) ? (s - t) + v : (v - t) + s;
    s = t;
  }
  hipmr_dd r = hipmr_two_sum_d(s, c);
  r = hipmr_block_reduce_pair<@@BLOCK@@>(r, [](hipmr_dd a, hipmr_dd b) { return hipmr_dd_add(a, b); });
  if (threadIdx.x == 0) {
    const double total = __builtin_isfinite(r.hi) ? r.hi + r.lo : r.hi;
    if constexpr (NORM && SCALED) *hipmr_out = hipmr_post * (sqrt(total) / *hipmr_scale64);
    else if constexpr (NORM) *hipmr_out = hipmr_post * sqrt(total);
    else *hipmr_out = hipmr_post * total;
  }
}
)HIP";



// ------------------------------------------------------------ batching
// Segments [off[s], off[s+1]) of the concatenated arrays are cut into tiles:
// tile 0 of a segment holds its unaligned head plus up to T body elements,
// later tiles T body elements each, where body elements start at the first
// index congruent to `head` modulo V (every accessed array is 16-byte aligned
// there) and T = 64 * V * IPT.  One wave reduces one tile.  The partition of
// a segment depends only on its bounds, V and IPT, never on other segments.
const char* kSegHelpers = R"HIP(
__device__ __forceinline__ void hipmr_seg_clamp(long long a0, long long b0, long long total,
                                                long long head, int V,
                                                long long& a, long long& b, long long& ab) {
  a = a0;
  b = b0;
  a = a < 0 ? 0 : (a > total ? total : a);
  b = b < a ? a : (b > total ? total : b);
  long long r = (head - a) % V;
  if (r < 0) r += V;
  ab = a + r < b ? a + r : b;
}
__device__ __forceinline__ void hipmr_seg_bounds(const long long* __restrict__ off, int s,
                                                 long long total, long long head, int V,
                                                 long long& a, long long& b, long long& ab) {
  hipmr_seg_clamp(off[s], off[s + 1], total, head, V, a, b, ab);
}
__device__ __forceinline__ int hipmr_seg_tiles(long long a, long long b, long long ab, long long T) {
  if (b == a) return 0;
  const long long t = (b - ab + T - 1) / T;
  return t < 1 ? 1 : (int)t;
}

// The tile table: tiles per segment and their exclusive prefix, by one block
// of B threads.  Each thread takes R consecutive segments per round of
// B * R (all offset loads issued before any is used).  Counts are summed in
// 64 bits and every entry is capped at the tile capacity of the workspace,
// so offsets that describe more tiles than it holds (overlapping segments)
// can never send a later kernel past it.  The table goes to `lds` and / or
// `glob` (either may be null); it is complete when this returns.
template <int B, int R = 4>
__device__ void hipmr_seg_plan(const long long* __restrict__ off, int nseg, long long total,
                               long long head, int V, long long T, long long cap,
                               int* lds, int* __restrict__ glob) {
  __shared__ long long hipmr_wsum[B / 64];
  __shared__ long long hipmr_carry;
  const auto hipmr_plus = [](long long p, long long q) { return p + q; };
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (threadIdx.x == 0) hipmr_carry = 0;
  __syncthreads();
  for (int base = 0; base < nseg; base += B * R) {
    const int s0 = base + threadIdx.x * R;
    long long o[R + 1];
#pragma unroll
    for (int j = 0; j <= R; ++j) o[j] = s0 + j <= nseg ? off[s0 + j] : 0;
    long long t[R], tsum = 0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      t[j] = 0;
      if (s0 + j < nseg) {
        long long a, b, ab;
        hipmr_seg_clamp(o[j], o[j + 1], total, head, V, a, b, ab);
        t[j] = hipmr_seg_tiles(a, b, ab, T);
      }
      tsum += t[j];
    }
    const long long x = hipmr_dpp_scan(tsum, 0LL, hipmr_plus);   // inclusive scan in the wave
    if (l == 63) hipmr_wsum[w] = x;
    __syncthreads();
    if (w == 0) {                                // scan of the wave totals
      const long long v = hipmr_dpp_scan(l < B / 64 ? hipmr_wsum[l] : 0LL, 0LL, hipmr_plus);
      if (l < B / 64) hipmr_wsum[l] = v;
    }
    __syncthreads();
    const long long excl = hipmr_carry + (w > 0 ? hipmr_wsum[w - 1] : 0) + x - tsum;
    long long run = excl;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      if (s0 + j < nseg) {
        const int v = (int)(run < cap ? run : cap);
        if (lds) lds[s0 + j] = v;
        if (glob) glob[s0 + j] = v;
      }
      run += t[j];
    }
    __syncthreads();
    if (threadIdx.x == B - 1) hipmr_carry = excl + tsum < cap ? excl + tsum : cap;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int v = (int)hipmr_carry;
    if (lds) lds[nseg] = v;
    if (glob) glob[nseg] = v;
  }
  __syncthreads();
}
)HIP";

// Planner (for tables too large for LDS): the tile table in global memory,
// one block of 1024 threads.
const char* kSegPlan = R"HIP(
extern "C" __global__ void __launch_bounds__(1024)
@@KNAME@@(const long long* __restrict__ hipmr_off, int hipmr_nseg, long long hipmr_total,
          long long hipmr_head, int* __restrict__ hipmr_tile_start, long long hipmr_cap)
{
  hipmr_seg_plan<1024>(hipmr_off, hipmr_nseg, hipmr_total, hipmr_head, @@VEC@@,
                       64LL * @@VEC@@ * @@IPT@@, hipmr_cap, nullptr, hipmr_tile_start);
}
)HIP";

// Persistent stage 1: waves take tiles t = wave, wave + nwaves, ...  (With
// the table in LDS this is also the planner: no separate planning launch.)
// Per tile, every load is issued before any result is used: the head and
// tail elements, then the body chunks; the next tile's segment is found (in
// the table) and its offsets fetched while they are in flight.  The wave's
// fold is a DPP scan whose last lane holds the tile partial.
const char* kSegS1 = R"HIP(
__device__ __forceinline__ hipmr_acc hipmr_wave_total(hipmr_acc v, hipmr_acc e, int lane) {
  if constexpr (sizeof(hipmr_acc) == 4 || sizeof(hipmr_acc) == 8) {
    return hipmr_dpp_scan(v, e, [](hipmr_acc a, hipmr_acc b) { return hipmr_combine(a, b); });
  } else {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const hipmr_acc y = __shfl_up(v, d, 64);
      if (lane >= d) v = hipmr_combine(y, v);
    }
    return v;
  }
}

extern "C" __global__ void __launch_bounds__(@@BLOCK@@)
@@KNAME@@(@@PARAMS@@, long long hipmr_total, long long hipmr_head,
          const long long* __restrict__ hipmr_offsets, int hipmr_nseg,
          int* __restrict__ hipmr_tile_start, hipmr_acc* __restrict__ hipmr_tpart,
          long long hipmr_cap)
{
  typedef @@IDX@@ hipmr_idx;
  constexpr int HIPMR_B = @@BLOCK@@, HIPMR_U = @@IPT@@, HIPMR_V = @@VEC@@, HIPMR_LDS_SEGS = @@LDS_SEGS@@;
  constexpr bool HIPMR_NTL = @@NTL@@, HIPMR_NTS = @@NTS@@;
  constexpr long long HIPMR_T = 64LL * HIPMR_V * HIPMR_U;
  const hipmr_idx n = (hipmr_idx)hipmr_total;
  const hipmr_acc hipmr_neutral = (hipmr_acc)(@@NEUTRAL@@);
  const int hipmr_lane = threadIdx.x & 63;
  // the tile-start table: a variant with LDS room computes it there in
  // every block (block 0 also writes it to global memory for the
  // per-segment fold); otherwise the planner has written it to global
  // memory.  (The host picks the LDS variant only when the table fits.)
  const int* hipmr_tab;
  if constexpr (HIPMR_LDS_SEGS > 0) {
    __shared__ int hipmr_ts_lds[HIPMR_LDS_SEGS > 0 ? HIPMR_LDS_SEGS : 1];
    if (hipmr_nseg >= HIPMR_LDS_SEGS) return;
    hipmr_seg_plan<HIPMR_B>(hipmr_offsets, hipmr_nseg, hipmr_total, hipmr_head, HIPMR_V, HIPMR_T,
                            hipmr_cap, hipmr_ts_lds, blockIdx.x == 0 ? hipmr_tile_start : nullptr);
    hipmr_tab = hipmr_ts_lds;
  } else {
    hipmr_tab = hipmr_tile_start;
  }
  // the planner caps the table at the workspace's tile capacity; the cap is
  // applied here again so that no tile partial is written past it
  const int hipmr_total_tiles = hipmr_tab[hipmr_nseg] < hipmr_cap ? hipmr_tab[hipmr_nseg] : (int)hipmr_cap;
  const int hipmr_nwaves = gridDim.x * (HIPMR_B / 64);
  // segment of a tile: the last s with tile_start[s] <= tile (64-way ballot search)
  auto hipmr_find = [&](int hipmr_tile) -> int {
    int hipmr_lo = 0, hipmr_hi = hipmr_nseg - 1;
    while (hipmr_lo < hipmr_hi) {
      const int hipmr_step = (hipmr_hi - hipmr_lo + 64) / 64;
      const int hipmr_cand = hipmr_lo + hipmr_lane * hipmr_step;
      const bool hipmr_pred = hipmr_cand <= hipmr_hi && hipmr_tab[hipmr_cand] <= hipmr_tile;
      const unsigned long long hipmr_m = __ballot(hipmr_pred);
      const int hipmr_k = 63 - __builtin_clzll(hipmr_m);
      hipmr_lo = hipmr_lo + hipmr_k * hipmr_step;
      hipmr_hi = hipmr_lo + hipmr_step - 1 < hipmr_hi ? hipmr_lo + hipmr_step - 1 : hipmr_hi;
    }
    return hipmr_lo;
  };
  int hipmr_t = blockIdx.x * (HIPMR_B / 64) + (threadIdx.x >> 6);
  int hipmr_s = 0;
  long long hipmr_oa = 0, hipmr_ob = 0;
  if (hipmr_t < hipmr_total_tiles) {
    hipmr_s = hipmr_find(hipmr_t);
    hipmr_oa = hipmr_offsets[hipmr_s];
    hipmr_ob = hipmr_offsets[hipmr_s + 1];
  }
  for (; hipmr_t < hipmr_total_tiles; hipmr_t += hipmr_nwaves) {
    long long hipmr_sa, hipmr_sb, hipmr_sab;
    hipmr_seg_clamp(hipmr_oa, hipmr_ob, hipmr_total, hipmr_head, HIPMR_V, hipmr_sa, hipmr_sb, hipmr_sab);
    const long long hipmr_k = hipmr_t - hipmr_tab[hipmr_s];
    const long long hipmr_tstart = hipmr_k == 0 ? hipmr_sa : hipmr_sab + hipmr_k * HIPMR_T;
    const long long hipmr_hend = hipmr_k == 0 ? hipmr_sab : hipmr_tstart;
    const long long hipmr_te = hipmr_sab + (hipmr_k + 1) * HIPMR_T < hipmr_sb ? hipmr_sab + (hipmr_k + 1) * HIPMR_T : hipmr_sb;
    const long long hipmr_nch = hipmr_te > hipmr_hend ? (hipmr_te - hipmr_hend) / HIPMR_V : 0;
    const long long hipmr_tail = hipmr_hend + hipmr_nch * HIPMR_V;
    // the unaligned head (tile 0 only) and the ragged tail, one element per lane
    hipmr_acc hipmr_hv = hipmr_neutral, hipmr_tv = hipmr_neutral;
    const bool hipmr_in_head = hipmr_lane < hipmr_hend - hipmr_tstart;
    const bool hipmr_in_tail = hipmr_lane < hipmr_te - hipmr_tail;
    if (hipmr_in_head) {
      const hipmr_idx i = (hipmr_idx)(hipmr_tstart + hipmr_lane);
      hipmr_hv = (hipmr_acc)(@@MAP@@);
    }
    if (hipmr_in_tail) {
      const hipmr_idx i = (hipmr_idx)(hipmr_tail + hipmr_lane);
      hipmr_tv = (hipmr_acc)(@@MAP@@);
    }
    hipmr_acc hipmr_a[HIPMR_U];
#pragma unroll
    for (int u = 0; u < HIPMR_U; ++u) hipmr_a[u] = hipmr_neutral;
    @@DECL_PACKS@@
    const bool hipmr_full = hipmr_nch == 64LL * HIPMR_U;   // every lane has all U chunks
    if (hipmr_full) {
#pragma unroll
      for (int hipmr_u = 0; hipmr_u < HIPMR_U; ++hipmr_u) {
        const long long hipmr_off = hipmr_hend + (hipmr_lane + 64LL * hipmr_u) * HIPMR_V;
        @@LOADS@@
      }
    } else {
#pragma unroll
      for (int hipmr_u = 0; hipmr_u < HIPMR_U; ++hipmr_u) {
        const long long hipmr_c = hipmr_lane + 64 * hipmr_u;
        if (hipmr_c < hipmr_nch) {
          const long long hipmr_off = hipmr_hend + hipmr_c * HIPMR_V;
          @@LOADS@@
        }
      }
    }
    const int hipmr_tn = hipmr_t + hipmr_nwaves;
    if (hipmr_tn < hipmr_total_tiles) {
      hipmr_s = hipmr_find(hipmr_tn);
      hipmr_oa = hipmr_offsets[hipmr_s];
      hipmr_ob = hipmr_offsets[hipmr_s + 1];
    }
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < HIPMR_U; ++hipmr_u) {
      const long long hipmr_c = hipmr_lane + 64 * hipmr_u;
      if (hipmr_full || hipmr_c < hipmr_nch) {
        const long long hipmr_off = hipmr_hend + hipmr_c * HIPMR_V;
#pragma unroll
        for (int hipmr_j = 0; hipmr_j < HIPMR_V; ++hipmr_j) {
          const hipmr_idx i = (hipmr_idx)(hipmr_off + hipmr_j);
          hipmr_a[hipmr_u] = hipmr_combine(hipmr_a[hipmr_u], (hipmr_acc)(@@VMAP@@));
        }
      }
    }
    // the head joins on the left of the body it precedes (combined only
    // now, so that no wait for its load comes before the body's loads)
    if (hipmr_in_head) hipmr_a[0] = hipmr_combine(hipmr_hv, hipmr_a[0]);
    if (hipmr_in_tail) hipmr_a[HIPMR_U - 1] = hipmr_combine(hipmr_a[HIPMR_U - 1], hipmr_tv);
    hipmr_acc hipmr_r = hipmr_fold<HIPMR_U>(hipmr_a);
    hipmr_r = hipmr_wave_total(hipmr_r, hipmr_neutral, hipmr_lane);
    if (hipmr_lane == 63) hipmr_tpart[hipmr_t] = hipmr_r;
  }
}
)HIP";

// Stage 2: one wave per segment folds its tile partials in tile order.
const char* kSegS2 = R"HIP(
extern "C" __global__ void __launch_bounds__(@@BLOCK@@)
@@KNAME@@(const int* __restrict__ hipmr_tile_start, int hipmr_nseg,
          const hipmr_acc* __restrict__ hipmr_tpart, hipmr_acc* __restrict__ hipmr_out,
          long long hipmr_cap)
{
  const int s = blockIdx.x * (@@BLOCK@@ / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (s >= hipmr_nseg) return;                  // whole waves only
  const hipmr_acc hipmr_neutral = (hipmr_acc)(@@NEUTRAL@@);
  hipmr_acc r = hipmr_neutral;
  const int t1 = hipmr_tile_start[s + 1] < hipmr_cap ? hipmr_tile_start[s + 1] : (int)hipmr_cap;
  // lane order t, t + 64, t + 128, ...; eight loads in flight per round
  for (int t = hipmr_tile_start[s] + lane; t < t1; t += 64 * 8) {
    hipmr_acc v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (t + 64 * k < t1) v[k] = hipmr_tpart[t + 64 * k];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (t + 64 * k < t1) r = hipmr_combine(r, v[k]);
  }
  r = hipmr_block_reduce<64>(r, hipmr_neutral);
  if (lane == 0) hipmr_out[s] = r;
}
)HIP";

// ------------------------------------------------------------ prefix scan
// Reduce-then-scan over a fixed partition: wave w owns the elements
// [head + w C, head + (w + 1) C) (wave 0 also the unaligned head [0, head)),
// C = P passes x U sub-tiles x 64 lanes x V elements; lane l owns the V
// consecutive elements at 64 V u + V l of each sub-tile.  Pass 1 folds each
// wave's range; pass 2 (one block) scans the wave totals; pass 3 rescans each
// range from its wave prefix.  The order of every combination is a fixed
// function of n and the geometry.
// Data-parallel-primitive (DPP) lane moves and the inclusive wave scan built
// from them (shared by the segmented and scan kernels).
const char* kDppHelpers = R"HIP(
// DPP lane moves on 32-bit halves: lanes whose source lies outside the
// pattern (or whose row is masked off) receive `fill`.
template <int CTRL, int ROWS, typename T>
__device__ __forceinline__ T hipmr_dpp(T v, T fill) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(
        __builtin_bit_cast(int, fill), __builtin_bit_cast(int, v), CTRL, ROWS, 0xf, false));
  } else {
    const unsigned long long a = __builtin_bit_cast(unsigned long long, v);
    const unsigned long long f = __builtin_bit_cast(unsigned long long, fill);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)f, (int)(unsigned)a, CTRL, ROWS, 0xf, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)(f >> 32), (int)(unsigned)(a >> 32),
                                                              CTRL, ROWS, 0xf, false);
    return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
  }
}

// inclusive scan across the wave of a 4- or 8-byte value under op (lane l
// receives v_0 op ... op v_l, the earlier lanes always on the left): shifts
// by 1, 2, 4, 8 inside each row of 16 lanes, then the totals of row 0 /
// rows 0-1 broadcast into the rows after them; e is op's neutral element
template <typename T, typename Op>
__device__ __forceinline__ T hipmr_dpp_scan(T v, T e, Op op) {
  v = op(hipmr_dpp<0x111, 0xf>(v, e), v);     // row_shr:1
  v = op(hipmr_dpp<0x112, 0xf>(v, e), v);     // row_shr:2
  v = op(hipmr_dpp<0x114, 0xf>(v, e), v);     // row_shr:4
  v = op(hipmr_dpp<0x118, 0xf>(v, e), v);     // row_shr:8
  v = op(hipmr_dpp<0x142, 0xa>(v, e), v);     // row_bcast:15 into rows 1, 3
  v = op(hipmr_dpp<0x143, 0xc>(v, e), v);     // row_bcast:31 into rows 2, 3
  return v;
}
)HIP";

const char* kScanHelpers = R"HIP(
// inclusive scan across the wave (lane l receives v_0 (+) ... (+) v_l)
template <typename T>
__device__ __forceinline__ T hipmr_wave_scan(T v, int lane, T e) {
  if constexpr (sizeof(T) == 4 || sizeof(T) == 8) {
    return hipmr_dpp_scan(v, e, [](T a, T b) { return hipmr_combine(a, b); });
  } else {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const T y = __shfl_up(v, d, 64);
      if (lane >= d) v = hipmr_combine(y, v);
    }
    return v;
  }
}
)HIP";

const char* kScanUp = R"HIP(
extern "C" __global__ void __launch_bounds__(@@BLOCK@@)
@@KNAME@@(@@PARAMS@@, long long hipmr_n, long long hipmr_head, int hipmr_passes,
          long long hipmr_waves, hipmr_acc* __restrict__ hipmr_partial)
{
  typedef @@IDX@@ hipmr_idx;
  constexpr int HIPMR_B = @@BLOCK@@, HIPMR_U = @@IPT@@, HIPMR_V = @@VEC@@;
  constexpr bool HIPMR_NTL = @@NTL@@, HIPMR_NTS = @@NTS@@;
  const hipmr_idx n = (hipmr_idx)hipmr_n;
  const hipmr_acc hipmr_neutral = (hipmr_acc)(@@NEUTRAL@@);
  const int hipmr_lane = threadIdx.x & 63;
  const long long hipmr_w = (long long)blockIdx.x * (HIPMR_B / 64) + (threadIdx.x >> 6);
  if (hipmr_w >= hipmr_waves) return;           // whole waves; no block barrier below
  const long long hipmr_h = hipmr_head < hipmr_n ? hipmr_head : hipmr_n;
  const long long hipmr_sub = 64LL * HIPMR_V;
  const long long hipmr_c = hipmr_sub * HIPMR_U * hipmr_passes;
  const long long hipmr_b0 = hipmr_h + hipmr_w * hipmr_c;
  const long long hipmr_e = hipmr_b0 + hipmr_c < hipmr_n ? hipmr_b0 + hipmr_c : hipmr_n;
  hipmr_acc hipmr_a[HIPMR_U];
#pragma unroll
  for (int u = 0; u < HIPMR_U; ++u) hipmr_a[u] = hipmr_neutral;
  if (hipmr_w == 0 && hipmr_lane < hipmr_h) {
    const hipmr_idx i = (hipmr_idx)hipmr_lane;
    hipmr_a[0] = hipmr_combine(hipmr_a[0], (hipmr_acc)(@@MAP@@));
  }
  for (int hipmr_p = 0; hipmr_p < hipmr_passes; ++hipmr_p) {
    const long long hipmr_pb = hipmr_b0 + (long long)hipmr_p * hipmr_sub * HIPMR_U;
    if (hipmr_pb >= hipmr_e) break;
    @@DECL_PACKS@@
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < HIPMR_U; ++hipmr_u) {
      const long long hipmr_off = hipmr_pb + hipmr_sub * hipmr_u + (long long)hipmr_lane * HIPMR_V;
      if (hipmr_off + HIPMR_V <= hipmr_e) {
        @@LOADS@@
      }
    }
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < HIPMR_U; ++hipmr_u) {
      const long long hipmr_off = hipmr_pb + hipmr_sub * hipmr_u + (long long)hipmr_lane * HIPMR_V;
      if (hipmr_off + HIPMR_V <= hipmr_e) {
#pragma unroll
        for (int hipmr_j = 0; hipmr_j < HIPMR_V; ++hipmr_j) {
          const hipmr_idx i = (hipmr_idx)(hipmr_off + hipmr_j);
          hipmr_a[hipmr_u] = hipmr_combine(hipmr_a[hipmr_u], (hipmr_acc)(@@VMAP@@));
        }
      } else {
        for (long long hipmr_k = hipmr_off; hipmr_k < hipmr_e; ++hipmr_k) {
          const hipmr_idx i = (hipmr_idx)hipmr_k;
          hipmr_a[hipmr_u] = hipmr_combine(hipmr_a[hipmr_u], (hipmr_acc)(@@MAP@@));
        }
      }
    }
  }
  hipmr_acc hipmr_r = hipmr_fold<HIPMR_U>(hipmr_a);
  hipmr_r = hipmr_block_reduce<64>(hipmr_r, hipmr_neutral);
  if (hipmr_lane == 0) hipmr_partial[hipmr_w] = hipmr_r;
}
)HIP";

// Pass 2, in two launches over the wave totals (coalesced, one per thread):
// every block of 1024 scans its 1024 totals (exclusive, within the block)
// and writes the block total; then one block scans the block totals.
const char* kScanMid = R"HIP(
template <int B>
__device__ __forceinline__ hipmr_acc hipmr_block_exclusive(hipmr_acc v, hipmr_acc neutral, hipmr_acc* total) {
  constexpr int W = B / 64;
  __shared__ hipmr_acc hipmr_wt[W];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const hipmr_acc x = hipmr_wave_scan(v, lane, neutral);
  if (lane == 63) hipmr_wt[w] = x;
  __syncthreads();
  if (w == 0) {
    hipmr_acc t = lane < W ? hipmr_wt[lane] : neutral;
    t = hipmr_wave_scan(t, lane, neutral);
    if (lane < W) hipmr_wt[lane] = t;
  }
  __syncthreads();
  const hipmr_acc up = __shfl_up(x, 1, 64);
  hipmr_acc r = lane == 0 ? neutral : up;
  if (w > 0) r = hipmr_combine(hipmr_wt[w - 1], r);
  *total = hipmr_wt[W - 1];
  return r;
}

extern "C" __global__ void __launch_bounds__(1024)
@@KNAME@@(const hipmr_acc* __restrict__ hipmr_partial, long long hipmr_waves,
          hipmr_acc* __restrict__ hipmr_prefix, hipmr_acc* __restrict__ hipmr_btot, int hipmr_top)
{
  const hipmr_acc hipmr_neutral = (hipmr_acc)(@@NEUTRAL@@);
  // hipmr_top == 0: block b scans totals [1024 b, 1024 b + 1024);
  // hipmr_top == 1: the single block scans the block totals in place
  const long long k = (long long)blockIdx.x * 1024 + threadIdx.x;
  const hipmr_acc* src = hipmr_top ? hipmr_btot : hipmr_partial;
  hipmr_acc* dst = hipmr_top ? hipmr_btot : hipmr_prefix;
  const long long count = hipmr_top ? (hipmr_waves + 1023) / 1024 : hipmr_waves;
  const hipmr_acc v = k < count ? src[k] : hipmr_neutral;
  hipmr_acc total;
  const hipmr_acc r = hipmr_block_exclusive<1024>(v, hipmr_neutral, &total);
  __syncthreads();                              // every read of src precedes the writes
  if (k < count) dst[k] = r;
  if (!hipmr_top && threadIdx.x == 0) hipmr_btot[blockIdx.x] = total;
}
)HIP";

// Pass 3: each wave rescans its range from its prefix and writes the outputs.
const char* kScanDown = R"HIP(
extern "C" __global__ void __launch_bounds__(@@BLOCK@@)
@@KNAME@@(@@PARAMS@@, long long hipmr_n, long long hipmr_head, int hipmr_passes,
          long long hipmr_waves, const hipmr_acc* __restrict__ hipmr_prefix,
          const hipmr_acc* __restrict__ hipmr_bpre, hipmr_acc* __restrict__ hipmr_out,
          int hipmr_exclusive)
{
  typedef @@IDX@@ hipmr_idx;
  constexpr int HIPMR_B = @@BLOCK@@, HIPMR_U = @@IPT@@, HIPMR_V = @@VEC@@;
  constexpr bool HIPMR_NTL = @@NTL@@, HIPMR_NTS = @@NTS@@;
  const hipmr_idx n = (hipmr_idx)hipmr_n;
  const hipmr_acc hipmr_neutral = (hipmr_acc)(@@NEUTRAL@@);
  const int hipmr_lane = threadIdx.x & 63;
  const long long hipmr_w = (long long)blockIdx.x * (HIPMR_B / 64) + (threadIdx.x >> 6);
  if (hipmr_w >= hipmr_waves) return;           // whole waves; no block barrier below
  const long long hipmr_h = hipmr_head < hipmr_n ? hipmr_head : hipmr_n;
  const long long hipmr_sub = 64LL * HIPMR_V;
  const long long hipmr_c = hipmr_sub * HIPMR_U * hipmr_passes;
  const long long hipmr_b0 = hipmr_h + hipmr_w * hipmr_c;
  const long long hipmr_e = hipmr_b0 + hipmr_c < hipmr_n ? hipmr_b0 + hipmr_c : hipmr_n;
  hipmr_acc hipmr_carry = hipmr_combine(hipmr_bpre[hipmr_w >> 10], hipmr_prefix[hipmr_w]);
  if (hipmr_w == 0 && hipmr_h > 0) {            // the unaligned head, one element per lane
    hipmr_acc hipmr_v = hipmr_neutral;
    if (hipmr_lane < hipmr_h) {
      const hipmr_idx i = (hipmr_idx)hipmr_lane;
      hipmr_v = (hipmr_acc)(@@MAP@@);
    }
    const hipmr_acc hipmr_x = hipmr_wave_scan(hipmr_v, hipmr_lane, hipmr_neutral);
    const hipmr_acc hipmr_up = __shfl_up(hipmr_x, 1, 64);
    if (hipmr_lane < hipmr_h)
      hipmr_out[hipmr_lane] = hipmr_exclusive ? (hipmr_lane == 0 ? hipmr_carry : hipmr_combine(hipmr_carry, hipmr_up))
                                              : hipmr_combine(hipmr_carry, hipmr_x);
    hipmr_carry = hipmr_combine(hipmr_carry, __shfl(hipmr_x, 63, 64));
  }
  for (int hipmr_p = 0; hipmr_p < hipmr_passes; ++hipmr_p) {
    const long long hipmr_pb = hipmr_b0 + (long long)hipmr_p * hipmr_sub * HIPMR_U;
    if (hipmr_pb >= hipmr_e) break;
    @@DECL_PACKS@@
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < HIPMR_U; ++hipmr_u) {
      const long long hipmr_off = hipmr_pb + hipmr_sub * hipmr_u + (long long)hipmr_lane * HIPMR_V;
      if (hipmr_off + HIPMR_V <= hipmr_e) {
        @@LOADS@@
      }
    }
    @@PASS_P@@
  }
}
)HIP";

// One pass of pass 3 over the chunks in registers (@@VMAPX@@ reads them):
// per sub-tile, the lane's inclusive prefixes of its V elements, a wave scan
// of the lane totals, the outputs, the carry.
const char* kScanDownPass = R"HIP(
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < HIPMR_U; ++hipmr_u) {
      const long long hipmr_off = hipmr_pb + hipmr_sub * hipmr_u + (long long)hipmr_lane * HIPMR_V;
      const bool hipmr_full = hipmr_off + HIPMR_V <= hipmr_e;
      hipmr_pack<hipmr_acc, HIPMR_V> hipmr_t;   // the lane's inclusive prefixes
      if (hipmr_full) {
#pragma unroll
        for (int hipmr_j = 0; hipmr_j < HIPMR_V; ++hipmr_j) {
          const hipmr_idx i = (hipmr_idx)(hipmr_off + hipmr_j);
          const hipmr_acc hipmr_m = (hipmr_acc)(@@VMAPX@@);
          hipmr_t.v[hipmr_j] = hipmr_j == 0 ? hipmr_m : hipmr_combine(hipmr_t.v[hipmr_j - 1], hipmr_m);
        }
      } else {
#pragma unroll
        for (int hipmr_j = 0; hipmr_j < HIPMR_V; ++hipmr_j) {
          hipmr_acc hipmr_m = hipmr_neutral;
          if (hipmr_off + hipmr_j < hipmr_e) {
            const hipmr_idx i = (hipmr_idx)(hipmr_off + hipmr_j);
            hipmr_m = (hipmr_acc)(@@MAP@@);
          }
          hipmr_t.v[hipmr_j] = hipmr_j == 0 ? hipmr_m : hipmr_combine(hipmr_t.v[hipmr_j - 1], hipmr_m);
        }
      }
      const hipmr_acc hipmr_x = hipmr_wave_scan(hipmr_t.v[HIPMR_V - 1], hipmr_lane, hipmr_neutral);
      const hipmr_acc hipmr_up = __shfl_up(hipmr_x, 1, 64);
      const hipmr_acc hipmr_pre = hipmr_lane == 0 ? hipmr_carry : hipmr_combine(hipmr_carry, hipmr_up);
      hipmr_pack<hipmr_acc, HIPMR_V> hipmr_o;
      if (hipmr_exclusive) {
        hipmr_o.v[0] = hipmr_pre;
#pragma unroll
        for (int hipmr_j = 1; hipmr_j < HIPMR_V; ++hipmr_j)
          hipmr_o.v[hipmr_j] = hipmr_combine(hipmr_pre, hipmr_t.v[hipmr_j - 1]);
      } else {
#pragma unroll
        for (int hipmr_j = 0; hipmr_j < HIPMR_V; ++hipmr_j)
          hipmr_o.v[hipmr_j] = hipmr_combine(hipmr_pre, hipmr_t.v[hipmr_j]);
      }
      if (hipmr_full) {
        hipmr_store<HIPMR_NTS>(hipmr_out + hipmr_off, hipmr_o);
      } else {
#pragma unroll
        for (int hipmr_j = 0; hipmr_j < HIPMR_V; ++hipmr_j)
          if (hipmr_off + hipmr_j < hipmr_e) hipmr_out[hipmr_off + hipmr_j] = hipmr_o.v[hipmr_j];
      }
      hipmr_carry = hipmr_combine(hipmr_carry, __shfl(hipmr_x, 63, 64));
    }
)HIP";

void replace_all(std::string& s, const std::string& key, const std::string& val) {
    size_t pos = 0;
    while ((pos = s.find(key, pos)) != std::string::npos) {
        s.replace(pos, key.size(), val);
        pos += val.size();
    }
}

std::string combine_body(DType r, const KernelSpec& spec) {
    bool fp = r == DT_F32 || r == DT_F64;
    switch (canonical_combine(spec.combine)) {
        case Combine::Sum: return "a + b";
        case Combine::Max: return fp ? "__builtin_elementwise_maximum(a, b)" : "(a > b ? a : b)";
        case Combine::Min: return fp ? "__builtin_elementwise_minimum(a, b)" : "(a < b ? a : b)";
        default: return spec.combine;
    }
}

}  // namespace

const char* device_prelude() { return kPrelude; }

std::string render(const Program& prog, const KernelSpec& spec, std::string* symbol) {
    const char* tmpl = nullptr;
    const char* tag = "";
    bool reduce = false;
    bool comp = false;       // compensated helpers
    DType acc = prog.sig.result;
    std::string combine = spec.combine;
    switch (spec.kind) {
        case KernelKind::EwVector:
            tmpl = prog.info.shifts.empty() ? kEwVector : kEwVectorShift;
            tag = "ew";
            break;
        case KernelKind::EwScalar: tmpl = kEwScalar; tag = "ews"; break;
        case KernelKind::RedS1Vector:
            tmpl = prog.info.shifts.empty() ? kRedS1Vector : kRedS1VectorShift;
            tag = "rs1";
            reduce = true;
            break;
        case KernelKind::RedS1Scalar: tmpl = kRedS1Scalar; tag = "rs1s"; reduce = true; break;
        case KernelKind::RedS2: tmpl = kRedS2; tag = "rs2"; reduce = true; break;
        case KernelKind::CompS1Vector:
            tmpl = kCompS1Vector; tag = spec.square ? "nrm2" : "csum"; comp = true; break;
        case KernelKind::CompS1Scalar:
            tmpl = kCompS1Scalar; tag = spec.square ? "nrm2s" : "csums"; comp = true; break;
        case KernelKind::CompS2: tmpl = kCompS2; tag = spec.norm ? "nrm2f" : "csumf"; comp = true; break;
        case KernelKind::AmaxS1Vector:
            tmpl = kRedS1Vector; tag = "amax"; reduce = true; acc = DT_F32; combine = "max"; break;
        case KernelKind::AmaxS1Scalar:
            tmpl = kRedS1Scalar; tag = "amaxs"; reduce = true; acc = DT_F32; combine = "max"; break;
        case KernelKind::SegPlan: tmpl = kSegPlan; tag = "segplan"; break;
        case KernelKind::SegS1: tmpl = kSegS1; tag = "seg1"; reduce = true; break;
        case KernelKind::SegS2: tmpl = kSegS2; tag = "seg2"; reduce = true; break;
        case KernelKind::ScanUpVector: tmpl = kScanUp; tag = "scu"; reduce = true; break;
        case KernelKind::ScanUpScalar: tmpl = kScanUp; tag = "scus"; reduce = true; break;
        case KernelKind::ScanMid: tmpl = kScanMid; tag = "scm"; reduce = true; break;
        case KernelKind::ScanDownVector: tmpl = kScanDown; tag = "scd"; reduce = true; break;
        case KernelKind::ScanDownScalar: tmpl = kScanDown; tag = "scds"; reduce = true; break;
    }
    const bool scan = spec.kind == KernelKind::ScanUpVector || spec.kind == KernelKind::ScanUpScalar ||
                      spec.kind == KernelKind::ScanMid || spec.kind == KernelKind::ScanDownVector ||
                      spec.kind == KernelKind::ScanDownScalar;
    // scalar scan kinds: one-element chunks read through the expression itself
    const bool scan_scalar = spec.kind == KernelKind::ScanUpScalar || spec.kind == KernelKind::ScanDownScalar;
    const bool seg = spec.kind == KernelKind::SegPlan || spec.kind == KernelKind::SegS1;
    const bool amax = spec.kind == KernelKind::AmaxS1Vector || spec.kind == KernelKind::AmaxS1Scalar;
    std::string body = tmpl;

    // parameters in declaration order
    std::string params;
    for (size_t k = 0; k < prog.sig.args.size(); ++k) {
        const ArgDecl& a = prog.sig.args[k];
        if (k) params += ", ";
        if (a.pointer) {
            params += std::string(a.is_const ? "const " : "") + dtype_device_name(a.dtype) +
                      "* __restrict__ " + a.name;
        } else {
            params += std::string("const ") + dtype_device_name(a.dtype) + " " + a.name;
        }
    }
    if (params.empty()) params = "int hipmr_unused";

    std::string decl_packs, loads, stores;
    for (const ArgDecl& a : prog.sig.args) {
        if (!chunked(a)) continue;
        if (a.dtype == DT_FP8 && !a.written && spec.vec >= 4)
            decl_packs += "hipmr_pack_fp8ro<HIPMR_V> hipmr_p_" + a.name + "[HIPMR_U]; ";
        else
            decl_packs += std::string("hipmr_pack<") + dtype_device_name(a.dtype) + ", HIPMR_V> hipmr_p_" +
                          a.name + "[HIPMR_U]; ";
        if (!a.write_only)
            loads += "hipmr_load<HIPMR_NTL>(hipmr_p_" + a.name + "[hipmr_u], " + a.name + " + hipmr_off); ";
        if (a.written)
            stores += "hipmr_store<HIPMR_NTS>(" + a.name + " + hipmr_off, hipmr_p_" + a.name + "[hipmr_u]); ";
    }

    // shifted reads (vector elementwise kernels): distances, packs and loads
    std::string shift_init, shift_packs, shift_loads;
    // (the other vector kernels read shifted elements directly, as written)
    const bool shifts = (spec.kind == KernelKind::EwVector || spec.kind == KernelKind::RedS1Vector) &&
                        !prog.info.shifts.empty();
    if (shifts) {
        std::string bounds = "long long hipmr_smin = 0, hipmr_smax = 0; ";
        for (size_t r = 0; r < prog.info.shifts.size(); ++r) {
            const ShiftRead& sr = prog.info.shifts[r];
            const ArgDecl& a = prog.sig.args[sr.arg];
            const std::string k = std::to_string(r);
            shift_init += "const long long hipmr_s" + k + " = (long long)" + sr.offset + "; ";
            bounds += "hipmr_smin = hipmr_s" + k + " < hipmr_smin ? hipmr_s" + k + " : hipmr_smin; ";
            bounds += "hipmr_smax = hipmr_s" + k + " > hipmr_smax ? hipmr_s" + k + " : hipmr_smax; ";
            shift_packs += std::string("hipmr_pack<") + dtype_device_name(a.dtype) + ", HIPMR_V> hipmr_q" + k +
                           "[HIPMR_U]; ";
            // the reduce kernel loads every chunk (clamped into the array);
            // the elementwise kernel loads only chunks it evaluates as vectors
            const std::string at = spec.kind == KernelKind::RedS1Vector
                                       ? "hipmr_clampv(hipmr_off, hipmr_s" + k + ", hipmr_n - HIPMR_V)"
                                       : "hipmr_off + hipmr_s" + k;
            shift_loads += "hipmr_loadu(hipmr_q" + k + "[hipmr_u], " + a.name + " + " + at + "); ";
        }
        shift_init += bounds;
    }
    replace_all(body, "@@SHIFT_INIT@@", shift_init);
    replace_all(body, "@@SHIFT_PACKS@@", shift_packs);
    replace_all(body, "@@SHIFT_LOADS@@", shift_loads);

    std::string scalar_text = join_tokens(prog.toks);
    std::string vector_text = scan_scalar ? scalar_text
                                          : vectorize_accesses(prog.toks, prog.sig,
                                                               shifts ? prog.info.shifts : std::vector<ShiftRead>{});
    if (scan_scalar) {
        decl_packs.clear();
        loads.clear();
    }
    if (spec.kind == KernelKind::ScanDownVector || spec.kind == KernelKind::ScanDownScalar) {
        std::string pass_p = kScanDownPass;
        replace_all(pass_p, "@@VMAPX@@", vector_text);
        replace_all(body, "@@PASS_P@@", pass_p);
    }

    replace_all(body, "@@PARAMS@@", params);
    replace_all(body, "@@DECL_PACKS@@", decl_packs);
    replace_all(body, "@@LOADS@@", loads);
    replace_all(body, "@@STORES@@", stores);
    replace_all(body, "@@STMT@@", scalar_text);
    replace_all(body, "@@VSTMT@@", vector_text);
    if (amax) {   // norm pass 1: |map| as float
        scalar_text = "fabsf((float)(" + scalar_text + "))";
        vector_text = "fabsf((float)(" + vector_text + "))";
    }
    replace_all(body, "@@MAP@@", scalar_text);
    replace_all(body, "@@VMAP@@", vector_text);
    replace_all(body, "@@NEUTRAL@@", amax ? "0.0f" : (spec.neutral.empty() ? "0" : spec.neutral));
    replace_all(body, "@@SQUARE@@", spec.square ? "true" : "false");
    replace_all(body, "@@RUNS@@", spec.exact_runs ? "true" : "false");
    replace_all(body, "@@NORM@@", spec.norm ? "true" : "false");
    replace_all(body, "@@SCALED@@", spec.scaled ? "true" : "false");
    replace_all(body, "@@SCALE_GAP@@", std::to_string(kScaleOffset - kAmaxOffset));
    replace_all(body, "@@LDS_SEGS@@", std::to_string(spec.lds_segs));
    replace_all(body, "@@IDX@@", spec.idx64 ? "long long" : "int");
    replace_all(body, "@@BLOCK@@", std::to_string(spec.block));
    replace_all(body, "@@IPT@@", std::to_string(spec.ipt));
    replace_all(body, "@@VEC@@", std::to_string(spec.vec));
    replace_all(body, "@@NTL@@", spec.nt_loads ? "true" : "false");
    replace_all(body, "@@NTS@@", spec.nt_stores ? "true" : "false");

    std::ostringstream src;
    src << "// generated by hipmr: " << tag << " kernel of \"" << prog.name << "\"\n";
    src << kPrelude;
    std::string cbody;
    if (reduce) {
        KernelSpec cs = spec;
        cs.combine = combine;
        cbody = combine_body(acc, cs);
        src << "typedef " << dtype_device_name(acc) << " hipmr_acc;\n";
        src << "__device__ __forceinline__ hipmr_acc hipmr_combine(hipmr_acc a, hipmr_acc b) "
               "{ return (hipmr_acc)(" << cbody << "); }\n";
        src << kReduceHelpers;
    }
    if (comp) src << kCompHelpers;
    if (seg || scan) src << kDppHelpers;
    if (seg) src << kSegHelpers;
    if (scan) src << kScanHelpers;
    if (shifts) src << kShiftHelpers;
    // the symbol carries a hash of the whole source (prelude and helpers
    // included), so any change to the generated code renames the kernel
    src << body;
    std::string text = src.str();
    std::string key = sha256_hex(text.data(), text.size());
    std::string sym = prog.name + "_" + tag + "_" + key.substr(0, 8);
    replace_all(text, "@@KNAME@@", sym);
    if (symbol) *symbol = sym;
    return text;
}

}  // namespace hipmr
