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
    if constexpr (NT) __builtin_nontemporal_store(tmp[k], d + k);
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
  constexpr int B = @@BLOCK@@, U = @@IPT@@, V = @@VEC@@;
  constexpr bool NTL = @@NTL@@, NTS = @@NTS@@;
  const hipmr_idx n = (hipmr_idx)hipmr_n;
  // elements [0, head) precede the first aligned chunk; [t0, n) is the ragged tail
  const long long hipmr_h = hipmr_head < hipmr_n ? hipmr_head : hipmr_n;
  const long long hipmr_nc = (hipmr_n - hipmr_h) / V;
  const long long hipmr_t0 = hipmr_h + hipmr_nc * V;
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
  const long long hipmr_step = (long long)gridDim.x * (B * U);
  long long hipmr_c0 = (long long)blockIdx.x * (B * U) + threadIdx.x;
  for (; hipmr_c0 + (U - 1) * B < hipmr_nc; hipmr_c0 += hipmr_step) {
    @@DECL_PACKS@@
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < U; ++hipmr_u) {
      const long long hipmr_off = hipmr_h + (hipmr_c0 + hipmr_u * B) * V;
      @@LOADS@@
    }
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < U; ++hipmr_u) {
      const long long hipmr_off = hipmr_h + (hipmr_c0 + hipmr_u * B) * V;
#pragma unroll
      for (int hipmr_j = 0; hipmr_j < V; ++hipmr_j) {
        const hipmr_idx i = (hipmr_idx)(hipmr_off + hipmr_j);
        { @@VSTMT@@; }
      }
      @@STORES@@
    }
  }
  if (hipmr_c0 < hipmr_nc) {
    @@DECL_PACKS@@
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < U; ++hipmr_u) {
      const long long hipmr_c = hipmr_c0 + hipmr_u * B;
      if (hipmr_c < hipmr_nc) {
        const long long hipmr_off = hipmr_h + hipmr_c * V;
        @@LOADS@@
      }
    }
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < U; ++hipmr_u) {
      const long long hipmr_c = hipmr_c0 + hipmr_u * B;
      if (hipmr_c < hipmr_nc) {
        const long long hipmr_off = hipmr_h + hipmr_c * V;
#pragma unroll
        for (int hipmr_j = 0; hipmr_j < V; ++hipmr_j) {
          const hipmr_idx i = (hipmr_idx)(hipmr_off + hipmr_j);
          { @@VSTMT@@; }
        }
        @@STORES@@
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
  constexpr int B = @@BLOCK@@, U = @@IPT@@, V = @@VEC@@;
  constexpr bool NTL = @@NTL@@, NTS = @@NTS@@;
  const hipmr_idx n = (hipmr_idx)hipmr_n;
  const hipmr_acc hipmr_neutral = (hipmr_acc)(@@NEUTRAL@@);
  hipmr_acc hipmr_a[U];
#pragma unroll
  for (int u = 0; u < U; ++u) hipmr_a[u] = hipmr_neutral;
  const long long hipmr_h = hipmr_head < hipmr_n ? hipmr_head : hipmr_n;
  const long long hipmr_nc = (hipmr_n - hipmr_h) / V;
  const long long hipmr_t0 = hipmr_h + hipmr_nc * V;
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
  const long long hipmr_step = (long long)gridDim.x * (B * U);
  long long hipmr_c0 = (long long)blockIdx.x * (B * U) + threadIdx.x;
  for (; hipmr_c0 + (U - 1) * B < hipmr_nc; hipmr_c0 += hipmr_step) {
    @@DECL_PACKS@@
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < U; ++hipmr_u) {
      const long long hipmr_off = hipmr_h + (hipmr_c0 + hipmr_u * B) * V;
      @@LOADS@@
    }
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < U; ++hipmr_u) {
      const long long hipmr_off = hipmr_h + (hipmr_c0 + hipmr_u * B) * V;
#pragma unroll
      for (int hipmr_j = 0; hipmr_j < V; ++hipmr_j) {
        const hipmr_idx i = (hipmr_idx)(hipmr_off + hipmr_j);
        hipmr_a[hipmr_u] = hipmr_combine(hipmr_a[hipmr_u], (hipmr_acc)(@@VMAP@@));
      }
    }
  }
  if (hipmr_c0 < hipmr_nc) {
    @@DECL_PACKS@@
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < U; ++hipmr_u) {
      const long long hipmr_c = hipmr_c0 + hipmr_u * B;
      if (hipmr_c < hipmr_nc) {
        const long long hipmr_off = hipmr_h + hipmr_c * V;
        @@LOADS@@
      }
    }
#pragma unroll
    for (int hipmr_u = 0; hipmr_u < U; ++hipmr_u) {
      const long long hipmr_c = hipmr_c0 + hipmr_u * B;
      if (hipmr_c < hipmr_nc) {
        const long long hipmr_off = hipmr_h + hipmr_c * V;
#pragma unroll
        for (int hipmr_j = 0; hipmr_j < V; ++hipmr_j) {
          const hipmr_idx i = (hipmr_idx)(hipmr_off + hipmr_j);
          hipmr_a[hipmr_u] = hipmr_combine(hipmr_a[hipmr_u], (hipmr_acc)(@@VMAP@@));
        }
      }
    }
  }
  hipmr_acc hipmr_r = hipmr_fold<U>(hipmr_a);
  hipmr_r = hipmr_block_reduce<B>(hipmr_r, hipmr_neutral);
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

void replace_all(std::string& s, const std::string& key, const std::string& val) {
    size_t pos = 0;
    while ((pos = s.find(key, pos)) != std::string::npos) {
        s.replace(pos, key.size(), val);
        pos += val.size();
    }
}

std::string combine_body(const Program& prog, const KernelSpec& spec) {
    DType r = prog.sig.result;
    bool fp = r == DT_F32 || r == DT_F64;
    switch (canonical_combine(spec.combine)) {
        case Combine::Sum: return "a + b";
        case Combine::Max: return fp ? "__builtin_elementwise_maximum(a, b)" : "(a > b ? a : b)";
        case Combine::Min: return fp ? "__builtin_elementwise_minimum(a, b)" : "(a < b ? a : b)";
        default: return spec.combine;
    }
}

}  // namespace

std::string render(const Program& prog, const KernelSpec& spec, std::string* symbol) {
    const char* tmpl = nullptr;
    const char* tag = "";
    bool reduce = false;
    switch (spec.kind) {
        case KernelKind::EwVector: tmpl = kEwVector; tag = "ew"; break;
        case KernelKind::EwScalar: tmpl = kEwScalar; tag = "ews"; break;
        case KernelKind::RedS1Vector: tmpl = kRedS1Vector; tag = "rs1"; reduce = true; break;
        case KernelKind::RedS1Scalar: tmpl = kRedS1Scalar; tag = "rs1s"; reduce = true; break;
        case KernelKind::RedS2: tmpl = kRedS2; tag = "rs2"; reduce = true; break;
    }
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
        if (!a.pointer || !(a.read || a.written)) continue;
        decl_packs += std::string("hipmr_pack<") + dtype_device_name(a.dtype) + ", V> hipmr_p_" +
                      a.name + "[U]; ";
        if (!a.write_only)
            loads += "hipmr_load<NTL>(hipmr_p_" + a.name + "[hipmr_u], " + a.name + " + hipmr_off); ";
        if (a.written)
            stores += "hipmr_store<NTS>(" + a.name + " + hipmr_off, hipmr_p_" + a.name + "[hipmr_u]); ";
    }

    std::string scalar_text = join_tokens(prog.toks);
    std::string vector_text = vectorize_accesses(prog.toks, prog.sig);

    replace_all(body, "@@PARAMS@@", params);
    replace_all(body, "@@DECL_PACKS@@", decl_packs);
    replace_all(body, "@@LOADS@@", loads);
    replace_all(body, "@@STORES@@", stores);
    replace_all(body, "@@STMT@@", scalar_text);
    replace_all(body, "@@VSTMT@@", vector_text);
    replace_all(body, "@@MAP@@", scalar_text);
    replace_all(body, "@@VMAP@@", vector_text);
    replace_all(body, "@@NEUTRAL@@", spec.neutral.empty() ? "0" : spec.neutral);
    replace_all(body, "@@IDX@@", spec.idx64 ? "long long" : "int");
    replace_all(body, "@@BLOCK@@", std::to_string(spec.block));
    replace_all(body, "@@IPT@@", std::to_string(spec.ipt));
    replace_all(body, "@@VEC@@", std::to_string(spec.vec));
    replace_all(body, "@@NTL@@", spec.nt_loads ? "true" : "false");
    replace_all(body, "@@NTS@@", spec.nt_stores ? "true" : "false");

    std::ostringstream src;
    src << "// generated by hipmr: " << tag << " kernel of \"" << prog.name << "\"\n";
    src << kPrelude;
    if (reduce) {
        src << "typedef " << dtype_device_name(prog.sig.result) << " hipmr_acc;\n";
        src << "__device__ __forceinline__ hipmr_acc hipmr_combine(hipmr_acc a, hipmr_acc b) "
               "{ return (hipmr_acc)(" << combine_body(prog, spec) << "); }\n";
        src << kReduceHelpers;
    }
    // the symbol carries a hash of everything that shapes the kernel
    std::string unnamed = (reduce ? combine_body(prog, spec) + "\n" : std::string()) + body;
    std::string key = sha256_hex(unnamed.data(), unnamed.size());
    std::string sym = prog.name + "_" + tag + "_" + key.substr(0, 8);
    replace_all(body, "@@KNAME@@", sym);
    src << body;
    if (symbol) *symbol = sym;
    return src.str();
}

}  // namespace hipmr
