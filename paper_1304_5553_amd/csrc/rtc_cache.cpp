// Run-time compilation with hipRTC and the compile cache.
//
// The paper's workflow (section "Core Method", compilation and caching
// figure): a source module goes through a cache lookup; on a miss the GPU
// compiler runs and its binary is stored; either way the binary is uploaded to
// the GPU and run.  Only kernels whose source changed are recompiled, so the
// others load near-instantly.  Here:
//   key     = SHA-256(source, compiler options, hipRTC version)
//   memory  = process-wide map (source, options, version) -> code object,
//             looked up by the text itself, so a hit costs one string hash
//             and one comparison, and the SHA-256 runs only on a miss
//   disk    = $HIPMR_CACHE_DIR/<key>.hsaco with a header (magic, payload size,
//             payload SHA-256) so that truncated or corrupted files are
//             detected and rebuilt; written to a temporary name and renamed
//   compile = hiprtcCompileProgram(--offload-arch=gfx950 -O3 -std=c++17)
//   upload  = hipModuleLoadData once per device, on first use there.
// Compilation never needs a GPU; module loading does.
#include <hip/hip_runtime_api.h>
#include <hip/hiprtc.h>
#include <sys/stat.h>
#include <unistd.h>

#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <unordered_map>

#include "common.h"

namespace hipmr {

constexpr int kMaxDevices = 64;

struct CodeObject {
    std::string key;
    std::string symbol;
    std::string image;
    std::mutex mu;
    hipModule_t module[kMaxDevices] = {};
    hipFunction_t function[kMaxDevices] = {};
};

namespace {

std::mutex g_mu;
std::unordered_map<std::string, std::shared_ptr<CodeObject>> g_cache;
std::atomic<uint64_t> g_mem_hits{0}, g_disk_hits{0}, g_compiles{0}, g_disk_rejects{0};
std::atomic<int64_t> g_compile_us{0};

const char kMagic[8] = {'H', 'I', 'P', 'M', 'R', 'C', 'O', '1'};

std::vector<std::string> compile_options() {
    const char* arch = std::getenv("HIPMR_ARCH");
    std::string a = std::string("--offload-arch=") + (arch && *arch ? arch : "gfx950");
    // -packed-fp32-ops: keep float code on the scalar-per-lane FP32 path
    return {a, "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
}

std::string compiler_version() {
    int major = 0, minor = 0;
    hiprtcVersion(&major, &minor);
    return "hiprtc-" + std::to_string(major) + "." + std::to_string(minor) + "-hip-" +
           std::to_string(HIP_VERSION);
}

void mkdir_p(const std::string& path) {
    std::string cur;
    for (size_t k = 0; k < path.size(); ++k) {
        cur += path[k];
        if (path[k] == '/' && cur.size() > 1) mkdir(cur.c_str(), 0755);
    }
    mkdir(path.c_str(), 0755);
}

std::string cache_dir() {
    const char* d = std::getenv("HIPMR_CACHE_DIR");
    if (d && *d) return d;
    const char* x = std::getenv("XDG_CACHE_HOME");
    if (x && *x) return std::string(x) + "/hipmr";
    const char* h = std::getenv("HOME");
    return std::string(h && *h ? h : "/tmp") + "/.cache/hipmr";
}

bool read_disk(const std::string& path, std::string* image) {
    FILE* f = std::fopen(path.c_str(), "rb");
    if (!f) return false;
    std::string data;
    char buf[1 << 16];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) data.append(buf, got);
    std::fclose(f);
    const size_t hdr = 8 + 8 + 64;
    if (data.size() < hdr || std::memcmp(data.data(), kMagic, 8) != 0) {
        g_disk_rejects++;
        return false;
    }
    uint64_t size;
    std::memcpy(&size, data.data() + 8, 8);
    if (size != data.size() - hdr) {
        g_disk_rejects++;
        return false;
    }
    std::string digest(data.data() + 16, 64);
    if (sha256_hex(data.data() + hdr, size) != digest) {
        g_disk_rejects++;
        return false;
    }
    *image = data.substr(hdr);
    return true;
}

void write_disk(const std::string& dir, const std::string& path, const std::string& image) {
    mkdir_p(dir);
    std::random_device rd;
    std::string tmp = path + ".tmp" + std::to_string(getpid()) + "_" + std::to_string(rd());
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return;   // the cache is an optimisation; failures to persist are silent
    uint64_t size = image.size();
    std::string digest = sha256_hex(image.data(), image.size());
    bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(&size, 1, 8, f) == 8 &&
              std::fwrite(digest.data(), 1, 64, f) == 64 &&
              std::fwrite(image.data(), 1, image.size(), f) == image.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) std::remove(tmp.c_str());
}

hipmr_status compile_source(const std::string& source, const std::vector<std::string>& opts,
                            std::string* image) {
    auto t0 = std::chrono::steady_clock::now();
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, source.c_str(), "hipmr_kernel.hip", 0, nullptr, nullptr) !=
        HIPRTC_SUCCESS)
        return fail(HIPMR_E_COMPILE, "hiprtcCreateProgram failed");
    std::vector<const char*> o;
    for (auto& s : opts) o.push_back(s.c_str());
    hiprtcResult r = hiprtcCompileProgram(prog, (int)o.size(), o.data());
    size_t log_size = 0;
    hiprtcGetProgramLogSize(prog, &log_size);
    std::string log(log_size, '\0');
    if (log_size) hiprtcGetProgramLog(prog, &log[0]);
    if (r != HIPRTC_SUCCESS) {
        hiprtcDestroyProgram(&prog);
        return fail(HIPMR_E_COMPILE, std::string("hipRTC: ") + hiprtcGetErrorString(r) + "\n" + log);
    }
    size_t code_size = 0;
    hiprtcGetCodeSize(prog, &code_size);
    image->assign(code_size, '\0');
    hiprtcGetCode(prog, &(*image)[0]);
    hiprtcDestroyProgram(&prog);
    g_compiles++;
    g_compile_us += std::chrono::duration_cast<std::chrono::microseconds>(
                        std::chrono::steady_clock::now() - t0).count();
    return HIPMR_OK;
}

}  // namespace

std::shared_ptr<CodeObject> get_or_build(const std::string& source, const std::string& symbol,
                                         hipmr_status* status) {
    static const std::vector<std::string> opts = compile_options();
    static const std::string version = compiler_version();
    std::string keytext = source;
    keytext += '\0';
    for (auto& o : opts) (keytext += o) += '\0';
    keytext += version;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_cache.find(keytext);
        if (it != g_cache.end()) {
            g_mem_hits++;
            *status = HIPMR_OK;
            return it->second;
        }
    }
    std::string key = sha256_hex(keytext.data(), keytext.size());
    auto co = std::make_shared<CodeObject>();
    co->key = key;
    co->symbol = symbol;
    std::string dir = cache_dir();
    std::string path = dir + "/" + key + ".hsaco";
    if (read_disk(path, &co->image)) {
        g_disk_hits++;
    } else {
        hipmr_status st = compile_source(source, opts, &co->image);
        if (st != HIPMR_OK) {
            *status = st;
            return nullptr;
        }
        write_disk(dir, path, co->image);
    }
    std::lock_guard<std::mutex> lk(g_mu);
    auto ins = g_cache.emplace(std::move(keytext), co);
    *status = HIPMR_OK;
    return ins.first->second;
}

hipmr_status get_function(CodeObject& co, void** fn) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(HIPMR_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(HIPMR_E_HIP, "device index out of range");
    std::lock_guard<std::mutex> lk(co.mu);
    if (!co.function[dev]) {
        if (capturing_now())
            return fail(HIPMR_E_INVALID, "kernel " + co.symbol + " is not loaded on this device yet: "
                                         "run the operation once before capturing it in a graph");
        if (no_alloc_now())
            return fail(HIPMR_E_INVALID, "kernel " + co.symbol + " is not loaded on this device yet: "
                                         "run the allocating entry point once on this device first");
        hipModule_t m;
        e = hipModuleLoadData(&m, co.image.data());
        if (e != hipSuccess)
            return fail(HIPMR_E_HIP, std::string("hipModuleLoadData: ") + hipGetErrorString(e));
        hipFunction_t f;
        e = hipModuleGetFunction(&f, m, co.symbol.c_str());
        if (e != hipSuccess) {
            (void)hipModuleUnload(m);
            return fail(HIPMR_E_HIP, "hipModuleGetFunction(" + co.symbol + "): " + hipGetErrorString(e));
        }
        co.module[dev] = m;
        co.function[dev] = f;
    }
    *fn = (void*)co.function[dev];
    return HIPMR_OK;
}

int device_cu_count() {
    static std::atomic<int> cus[kMaxDevices];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 256;
    int c = cus[dev].load();
    if (c == 0) {
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            c <= 0)
            c = 256;
        cus[dev].store(c);
    }
    return c;
}

hipmr_status launch(void* fn, unsigned grid, unsigned block, void** params, void* stream) {
    hipError_t e = hipModuleLaunchKernel((hipFunction_t)fn, grid, 1, 1, block, 1, 1, 0,
                                         (hipStream_t)stream, params, nullptr);
    if (e != hipSuccess)
        return fail(HIPMR_E_HIP, std::string("hipModuleLaunchKernel: ") + hipGetErrorString(e));
    return HIPMR_OK;
}

const std::string& code_object_symbol(const CodeObject& co) { return co.symbol; }
const std::string& code_object_image(const CodeObject& co) { return co.image; }

void cache_stats(hipmr_cache_stats* out) {
    out->memory_hits = g_mem_hits.load();
    out->disk_hits = g_disk_hits.load();
    out->compiles = g_compiles.load();
    out->disk_rejects = g_disk_rejects.load();
    out->compile_ms = g_compile_us.load() / 1000.0;
}

void cache_drop_memory() {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache.clear();
}

}  // namespace hipmr
