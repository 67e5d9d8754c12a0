// First-pass row plans compiled at run time.  The library carries compiled-in
// kernels for the general stages and for a few fixed radix sequences; any
// other sequence the planner picks can get its own RowPlan<R...> kernel
// (constant stage sizes, per-stage twiddle tables) compiled by hipRTC from
// the same header the library was built from (rsf_pass_a.h beside the
// library, checked against the hash recorded at build time), loaded as a
// module on the current device and cached on disk.  Anything missing (the
// headers, hipRTC, a compile error) leaves the general stages in use: this
// is a faster kernel for the same arithmetic, never a different result path.
#include <dlfcn.h>
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <sys/stat.h>
#include <unistd.h>

#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "rsf_launch.h"

#ifndef RSF_ROW_SRC_HASH
#define RSF_ROW_SRC_HASH 0ull
#endif
#ifndef RSF_OFFLOAD_ARCH
#define RSF_OFFLOAD_ARCH "gfx950"
#endif

namespace rsf {

namespace {

// the headers a row kernel is compiled from, in the order of the build's hash
const char* const kRowHeaders[] = {"rsf_pass_a.h", "rsf_device.h", "rsf_spill.h", "rsf_params.h"};

uint64_t fnv1a(const std::string& s, uint64_t h) {
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

bool read_file(const std::string& path, std::string* out) {
    std::ifstream f(path, std::ios::binary);
    if (!f) return false;
    std::ostringstream ss;
    ss << f.rdbuf();
    *out = ss.str();
    return true;
}

struct RtcState {
    bool ok = false;
    std::string csrc, rocm, cache;
    uint64_t src_hash = 0;
};

// Resolved once: the csrc directory beside this library with the headers it
// was built from, and RSF_RTC not "0".
const RtcState& rtc_state() {
    static RtcState st;
    static std::once_flag once;
    std::call_once(once, [] {
        const char* env = getenv("RSF_RTC");
        if (env && env[0] == '0') return;
        Dl_info info{};
        if (!dladdr((const void*)&rtc_state, &info) || !info.dli_fname) return;
        std::string lib = info.dli_fname;
        const size_t slash = lib.rfind('/');
        st.csrc = (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) + "/csrc";
        uint64_t h = 1469598103934665603ull;
        for (const char* name : kRowHeaders) {
            std::string text;
            if (!read_file(st.csrc + "/" + name, &text)) return;
            h = fnv1a(text, h);
        }
        if (h != (uint64_t)RSF_ROW_SRC_HASH) return;
        st.src_hash = h;
        const char* rocm = getenv("ROCM_PATH");
        st.rocm = rocm && rocm[0] ? rocm : "/opt/rocm";
        const char* c = getenv("RSF_KERNEL_CACHE");
        if (c && c[0]) {
            st.cache = c;
        } else {
            const char* xdg = getenv("XDG_CACHE_HOME");
            const char* home = getenv("HOME");
            st.cache = xdg && xdg[0] ? std::string(xdg) + "/rsfstat"
                       : home && home[0] ? std::string(home) + "/.cache/rsfstat"
                                         : std::string("/tmp/rsfstat-kernels");
        }
        st.ok = true;
    });
    return st;
}

void make_dirs(const std::string& path) {
    for (size_t i = 1; i <= path.size(); ++i)
        if (i == path.size() || path[i] == '/') (void)mkdir(path.substr(0, i).c_str(), 0755);
}

// A cached code object: "RSFROW1", the two kernel names, the byte count,
// then the bytes.
bool cache_read(const std::string& path, std::string names[2], std::string* code) {
    std::ifstream f(path, std::ios::binary);
    if (!f) return false;
    std::string magic;
    size_t n = 0;
    if (!std::getline(f, magic) || magic != "RSFROW1" || !std::getline(f, names[0]) || !std::getline(f, names[1]))
        return false;
    std::string count;
    if (!std::getline(f, count)) return false;
    n = (size_t)strtoull(count.c_str(), nullptr, 10);
    code->resize(n);
    f.read(&(*code)[0], (std::streamsize)n);
    return (size_t)f.gcount() == n && n > 0;
}

void cache_write(const std::string& dir, const std::string& path, const std::string names[2], const std::string& code) {
    make_dirs(dir);
    const std::string tmp = path + ".tmp." + std::to_string((long long)getpid());
    {
        std::ofstream f(tmp, std::ios::binary);
        if (!f) return;
        f << "RSFROW1\n" << names[0] << "\n" << names[1] << "\n" << code.size() << "\n";
        f.write(code.data(), (std::streamsize)code.size());
        if (!f) {
            (void)unlink(tmp.c_str());
            return;
        }
    }
    if (rename(tmp.c_str(), path.c_str()) != 0) (void)unlink(tmp.c_str());
}

bool compile(const RtcState& st, const std::string exprs[2], std::string names[2], std::string* code) {
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, "#include \"rsf_pass_a.h\"\n", "rsf_row_plan.hip", 0, nullptr, nullptr) !=
        HIPRTC_SUCCESS)
        return false;
    bool ok = hiprtcAddNameExpression(prog, exprs[0].c_str()) == HIPRTC_SUCCESS &&
              hiprtcAddNameExpression(prog, exprs[1].c_str()) == HIPRTC_SUCCESS;
    const std::string inc = "-I" + st.csrc, inc_hip = "-I" + st.rocm + "/include";
    const char* opts[] = {"--offload-arch=" RSF_OFFLOAD_ARCH, "-O3", "-std=c++17", inc.c_str(), inc_hip.c_str(),
                          // no packed FP32 instructions, as in the library's own device code
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    ok = ok && hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts) == HIPRTC_SUCCESS;
    if (!ok && getenv("RSF_RTC_VERBOSE")) {
        size_t log_n = 0;
        if (hiprtcGetProgramLogSize(prog, &log_n) == HIPRTC_SUCCESS && log_n > 1) {
            std::string log(log_n, '\0');
            if (hiprtcGetProgramLog(prog, &log[0]) == HIPRTC_SUCCESS)
                fprintf(stderr, "rsfstat: row plan %s not compiled:\n%s\n", exprs[0].c_str(), log.c_str());
        }
    }
    size_t n = 0;
    ok = ok && hiprtcGetCodeSize(prog, &n) == HIPRTC_SUCCESS && n > 0;
    if (ok) {
        code->resize(n);
        ok = hiprtcGetCode(prog, &(*code)[0]) == HIPRTC_SUCCESS;
    }
    for (int i = 0; ok && i < 2; ++i) {
        const char* low = nullptr;
        ok = hiprtcGetLoweredName(prog, exprs[i].c_str(), &low) == HIPRTC_SUCCESS && low;
        if (ok) names[i] = low;
    }
    (void)hiprtcDestroyProgram(&prog);
    return ok;
}

struct Loaded {
    bool tried = false;
    hipModule_t mod = nullptr;
    hipFunction_t fn[2] = {nullptr, nullptr};
};
std::mutex g_mu;
std::map<std::string, Loaded> g_loaded;

}  // namespace

bool row_plan_kernels(int order, const FftStages& plan, void* fn[2]) {
    fn[0] = fn[1] = nullptr;
    const RtcState& st = rtc_state();
    if (!st.ok || order < 1 || order > 3 || plan.n_stages < 2 || plan.n_stages > kMaxStages) return false;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return false;
    std::string radices;
    for (int i = 0; i < plan.n_stages; ++i) radices += (i ? ", " : "") + std::to_string(plan.radix[i]);
    std::string exprs[2];
    for (int nt = 0; nt < 2; ++nt)
        exprs[nt] = "rsf::rsf_fft_pass_a_k<" + std::to_string(order) + ", " + (nt ? "true" : "false") +
                    ", rsf::RowPlan<" + radices + ">>";
    const std::string key = std::to_string(device) + ":" + exprs[0];
    std::lock_guard<std::mutex> lock(g_mu);
    Loaded& e = g_loaded[key];
    if (!e.tried) {
        e.tried = true;
        char hex[17];
        snprintf(hex, sizeof hex, "%016llx",
                 (unsigned long long)fnv1a(exprs[0] + "|" + RSF_OFFLOAD_ARCH, st.src_hash));
        const std::string path = st.cache + "/row_" + hex + ".co";
        // a cached code object first; one that does not load (truncated,
        // another toolchain's) is replaced by a fresh compile
        auto load = [&](const std::string names[2], const std::string& code) {
            hipModule_t mod = nullptr;
            hipFunction_t f0 = nullptr, f1 = nullptr;
            if (hipModuleLoadData(&mod, code.data()) != hipSuccess) return false;
            if (hipModuleGetFunction(&f0, mod, names[0].c_str()) != hipSuccess ||
                hipModuleGetFunction(&f1, mod, names[1].c_str()) != hipSuccess) {
                (void)hipModuleUnload(mod);
                return false;
            }
            e.mod = mod;
            e.fn[0] = f0;
            e.fn[1] = f1;
            return true;
        };
        std::string names[2], code;
        const bool cached = cache_read(path, names, &code);
        if (!cached || !load(names, code)) {
            if (cached) (void)unlink(path.c_str());
            if (!compile(st, exprs, names, &code) || !load(names, code)) return false;
            cache_write(st.cache, path, names, code);
        }
    }
    if (!e.mod) return false;
    fn[0] = (void*)e.fn[0];
    fn[1] = (void*)e.fn[1];
    return true;
}

}  // namespace rsf
