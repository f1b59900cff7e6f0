// Run-time compilation and the process-wide cache of compiled kernels.
//
// The run-time compiler is the ROCm installation's hipRTC, loaded into a
// link-map namespace of its own (dlmopen).  A process may already hold
// another hipRTC under the same soname (PyTorch wheels bundle one, with an
// older compiler); a plain link or dlopen would bind to that copy, and its
// code for the same source can be markedly slower.
#include "rtc.h"

#include <dlfcn.h>
#include <hip/hiprtc.h>

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "qcw_common.h"

#ifndef QCW_ROCM_LIB
#define QCW_ROCM_LIB "/opt/rocm/lib"
#endif

namespace qcw {

namespace {

struct Api {
  decltype(&hiprtcCreateProgram) create;
  decltype(&hiprtcDestroyProgram) destroy;
  decltype(&hiprtcCompileProgram) compile;
  decltype(&hiprtcGetProgramLogSize) log_size;
  decltype(&hiprtcGetProgramLog) log;
  decltype(&hiprtcGetCodeSize) code_size;
  decltype(&hiprtcGetCode) code;
  decltype(&hiprtcGetErrorString) error_string;
  decltype(&hiprtcVersion) version;
  int ver;          // major * 100 + minor; 0 when unavailable
  std::string why;  // why loading failed
};

const Api &api() {
  static Api a{};
  static std::once_flag once;
  std::call_once(once, [] {
    const char *path = QCW_ROCM_LIB "/libhiprtc.so.7";
    void *h = dlmopen(LM_ID_NEWLM, path, RTLD_NOW | RTLD_LOCAL);
    if (!h) {
      const char *e = dlerror();
      a.why = std::string("cannot load ") + path + ": " + (e ? e : "?");
      return;
    }
    bool ok = true;
    auto sym = [&](auto &f, const char *name) {
      f = reinterpret_cast<std::remove_reference_t<decltype(f)>>(dlsym(h, name));
      ok = ok && f != nullptr;
    };
    sym(a.create, "hiprtcCreateProgram");
    sym(a.destroy, "hiprtcDestroyProgram");
    sym(a.compile, "hiprtcCompileProgram");
    sym(a.log_size, "hiprtcGetProgramLogSize");
    sym(a.log, "hiprtcGetProgramLog");
    sym(a.code_size, "hiprtcGetCodeSize");
    sym(a.code, "hiprtcGetCode");
    sym(a.error_string, "hiprtcGetErrorString");
    sym(a.version, "hiprtcVersion");
    int major = 0, minor = 0;
    if (!ok || a.version(&major, &minor) != HIPRTC_SUCCESS) {
      a = Api{};
      a.why = std::string(path) + " lacks the hipRTC entry points";
      return;
    }
    a.ver = major * 100 + minor;
  });
  return a;
}

struct Entry {
  hipModule_t mod = nullptr;
  RtcKernel k{};
};

std::mutex g_mu;
std::map<std::tuple<int, std::string, std::string>, std::unique_ptr<Entry>> g_cache;

int compile(const std::string &src, const char *name, std::vector<char> *code) {
  const Api &A = api();
  if (!A.ver) return fail(QCW_EHIP, "run-time compiler unavailable: %s", A.why.c_str());
  hiprtcProgram p = nullptr;
  if (A.create(&p, src.c_str(), "qcw_rtc.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
    return fail(QCW_EHIP, "hiprtcCreateProgram failed for %s", name);
  // The library's own flags: gfx950, no packed FP32 instructions, no
  // wave-level combining of atomics (a drawn ticket is used a tile later),
  // no contraction beyond the explicit fused multiply-adds.
  const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                        "-mllvm", "-amdgpu-atomic-optimizer-strategy=None"};
  const hiprtcResult rc = A.compile(p, (int)(sizeof(opts) / sizeof(opts[0])), opts);
  if (rc != HIPRTC_SUCCESS) {
    size_t n = 0;
    std::string log;
    if (A.log_size(p, &n) == HIPRTC_SUCCESS && n > 1) {
      log.resize(n);
      (void)A.log(p, &log[0]);
    }
    (void)A.destroy(&p);
    return fail(QCW_EHIP, "run-time compile of %s failed (%s): %.400s", name, A.error_string(rc),
                log.c_str());
  }
  size_t n = 0;
  if (A.code_size(p, &n) != HIPRTC_SUCCESS || n == 0) {
    (void)A.destroy(&p);
    return fail(QCW_EHIP, "run-time compile of %s gave no code", name);
  }
  code->resize(n);
  const hiprtcResult rg = A.code(p, code->data());
  (void)A.destroy(&p);
  if (rg != HIPRTC_SUCCESS) return fail(QCW_EHIP, "hiprtcGetCode failed for %s", name);
  return QCW_OK;
}

}  // namespace

int rtc_compiler_version() { return api().ver; }

int rtc_compile(const std::string &src, const char *name, size_t *code_bytes) {
  std::vector<char> code;
  const int rc = compile(src, name, &code);
  *code_bytes = rc ? 0 : code.size();
  return rc;
}

int rtc_get(const std::string &src, const char *name, const RtcKernel **out) {
  *out = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QCW_EHIP, "no current device");
  }
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_tuple(dev, src, std::string(name));
  auto it = g_cache.find(key);
  if (it != g_cache.end()) {
    *out = &it->second->k;
    return QCW_OK;
  }
  std::vector<char> code;
  int rc = compile(src, name, &code);
  if (rc) return rc;
  std::unique_ptr<Entry> e(new Entry());
  if (hipModuleLoadData(&e->mod, code.data()) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QCW_EHIP, "loading the compiled %s failed", name);
  }
  if (hipModuleGetFunction(&e->k.fn, e->mod, name) != hipSuccess ||
      hipFuncGetAttribute(&e->k.num_regs, HIP_FUNC_ATTRIBUTE_NUM_REGS, e->k.fn) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipModuleUnload(e->mod);
    return fail(QCW_EHIP, "compiled %s has no usable entry", name);
  }
  *out = &e->k;
  g_cache.emplace(std::move(key), std::move(e));
  return QCW_OK;
}

}  // namespace qcw
