// Internal declarations shared by the host-side translation units of
// libhipmr.so.  Device code lives only in the generated sources (see
// codegen.cpp); this header is host C++17.
#pragma once

#include <cstddef>
#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "hipmr.h"

namespace hipmr {

// ---------------------------------------------------------------- errors
// Thread-local last-error message plus status code helpers.
hipmr_status fail(hipmr_status code, const std::string& msg);
void clear_error();
const char* last_error();

// ---------------------------------------------------------------- dtypes
enum DType : int32_t {
    DT_NONE = 0,
    DT_F32 = HIPMR_F32, DT_F64 = HIPMR_F64, DT_I8 = HIPMR_I8, DT_U8 = HIPMR_U8,
    DT_I16 = HIPMR_I16, DT_U16 = HIPMR_U16, DT_I32 = HIPMR_I32, DT_U32 = HIPMR_U32,
    DT_I64 = HIPMR_I64, DT_BF16 = HIPMR_BF16, DT_F16 = HIPMR_F16, DT_FP8 = HIPMR_FP8,
    DT_C64 = HIPMR_C64,
};

int dtype_size(DType t);
const char* dtype_device_name(DType t);   // spelling used in generated device code
bool dtype_is_float(DType t);             // value type after a read is float or double
bool dtype_is_lowp(DType t);              // bf16 / f16 / fp8 storage types

// ---------------------------------------------------------------- front end
struct ArgDecl {
    std::string name;
    DType dtype = DT_NONE;
    bool pointer = false;
    bool is_const = false;
    // filled by the classifier
    bool read = false;        // the expression reads name[...] (or the scalar)
    bool written = false;     // the expression assigns name[i]
    bool write_only = false;  // written unconditionally before any read: no load needed
    bool lane = false;        // accessed as name[i]
    bool uniform = false;     // read as name[<integer literal>] (the same element for every i)
    bool shifted = false;     // read as name[i + E] / name[i - E], E uniform (see ShiftRead)
    bool other = false;       // accessed at any other index (or used as a bare pointer)
};

// An array the vector kernels move in 16-byte chunks (accessed as name[i] or
// written); arrays read only at constant indices are read directly instead.
inline bool chunked(const ArgDecl& a) { return a.pointer && (a.lane || a.written); }

struct Signature {
    bool is_reduce = false;
    DType result = DT_NONE;
    std::vector<ArgDecl> args;
};

// "[result_type ':'] decl (',' decl)*"
hipmr_status parse_signature(const std::string& text, Signature* out);

struct Token {
    enum Kind { Ident, Number, Punct, End } kind;
    std::string text;
    size_t pos;
};

hipmr_status lex(const std::string& src, std::vector<Token>* out);

// A read of an array at a fixed distance from the formal index, name[i + E]
// or name[i - E]: E holds only literals, scalar arguments, n, + - * / % and
// parentheses, so the distance is the same for every i.  The vector
// elementwise and plain reduce kernels load such reads as (unaligned) chunks;
// the other vector kernels read them element by element, as written.
struct ShiftRead {
    size_t arg;                 // index of the array in the signature
    std::string offset;         // C expression of the signed distance, "(0 + E)" / "(0 - E)"
};

struct ExprInfo {
    bool vectorizable = true;   // every array reference is name[i], a read of a fixed element
                                // or a shifted read of an array the expression does not write
    bool has_writes = false;
    std::vector<ShiftRead> shifts;   // distinct shifted reads, in order of appearance
};

// Classifies an elementwise statement list or a map expression against the
// signature: which arrays are read / written / write-only, and whether the
// lane-vectorised kernel applies.  Fills sig->args[*].read/written/write_only.
hipmr_status classify(const std::vector<Token>& toks, Signature* sig, bool is_map, ExprInfo* out);

// Source text of a token list (tokens separated by blanks).
std::string join_tokens(const std::vector<Token>& toks);

// Rewrites every array access name[i] into the register form used by the
// vector kernels: <name>_p[hipmr_u].v[hipmr_j].
std::string vectorize_accesses(const std::vector<Token>& toks, const Signature& sig,
                               const std::vector<ShiftRead>& shifts = {});

// Canonical combine operations (see hipmr_reduce).
enum class Combine { Sum, Max, Min, Generic };
Combine canonical_combine(const std::string& combine);

// ---------------------------------------------------------------- geometry
struct LaunchCfg {
    int block = 256;
    int ipt = 4;          // vector chunks per thread per pass
    int grid = 0;         // 0: derived
    int blocks_per_cu = 8;
    int vec = 0;          // 0: derived
    bool nt_loads = true;   // streaming (non-temporal) loads
    bool nt_stores = true;  // streaming (non-temporal) stores
    bool force_scalar = false;
    bool seg_global = false;  // segmented: tile table in global memory
};

// ---------------------------------------------------------------- codegen
enum class KernelKind : int32_t {
    EwVector = 0, EwScalar = 1, RedS1Vector = 2, RedS1Scalar = 3, RedS2 = 4,
    CompS1Vector = 5, CompS1Scalar = 6, CompS2 = 7, AmaxS1Vector = 8, AmaxS1Scalar = 9,
    SegPlan = 11, SegS1 = 12, SegS2 = 13,
    ScanUpVector = 14, ScanUpScalar = 15, ScanMid = 16, ScanDownVector = 17, ScanDownScalar = 18,
};

struct KernelSpec {
    KernelKind kind;
    bool idx64 = false;       // 64-bit formal index
    int block = 256;
    int ipt = 4;
    int vec = 4;
    bool nt_loads = true;
    bool nt_stores = true;
    std::string combine;      // reduce kinds
    std::string neutral;
    // precision extension
    bool square = false;      // CompS1: accumulate map^2 (norm)
    bool scaled = false;      // CompS1 / CompS2: apply the device-side power-of-two scale
    bool exact_runs = false;  // CompS1: map is one FP8 load; sum runs of <= 64 exactly
    bool norm = false;        // CompS2: finish as sqrt(sum) / scale
    // batching extension
    int lds_segs = 0;         // SegS1: tile-start table held in LDS (capacity), 0 = global
};

struct Program {                 // everything codegen needs about one handle
    std::string name;            // symbol prefix
    std::string expr;            // user text
    std::vector<Token> toks;
    Signature sig;
    ExprInfo info;
};

// Device helpers every generated module starts with (storage formats, chunk
// loads and stores).
const char* device_prelude();

// Renders the full device source (prelude + one kernel) and its symbol name.
std::string render(const Program& prog, const KernelSpec& spec, std::string* symbol);

// ---------------------------------------------------------------- RTC cache
struct CodeObject;   // opaque: compiled image + per-device modules/functions

// Compiles (or loads from the memory / disk cache) a source; never touches
// the GPU.  Returns nullptr with last_error set on failure.
std::shared_ptr<CodeObject> get_or_build(const std::string& source, const std::string& symbol,
                                         hipmr_status* status);

const std::string& code_object_symbol(const CodeObject& co);
const std::string& code_object_image(const CodeObject& co);

// hipFunction_t (as void*) of the code object on the current device; loads the
// module on first use on that device.
hipmr_status get_function(CodeObject& co, void** fn);

std::string sha256_hex(const void* data, size_t len);

// Current device's CU count (cached per device); 256 if it cannot be queried.
int device_cu_count();

hipmr_status launch(void* fn, unsigned grid, unsigned block, void** params, void* stream);

void cache_stats(hipmr_cache_stats* out);
void cache_drop_memory();

// True between hipmr_graph_begin_capture and hipmr_graph_end_capture on this
// thread: code objects must already be loaded then.
bool capturing_now();
// true while a no-allocation entry point runs on this thread: variants are
// neither built nor loaded then (only those already on the device are used)
bool no_alloc_now();
void set_no_alloc(bool on);

}  // namespace hipmr
