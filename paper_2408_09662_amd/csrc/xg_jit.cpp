// Runtime compilation of generated HIP source for gfx950 (hiprtc), with an
// on-disk code-object cache keyed by a hash of source, options and compiler
// version.  The paper compiles its generated file once, offline, with the
// vendor toolkit; here compilation happens at first use and is reused from
// the cache afterwards, so a program is compiled once per machine image.
#include <dlfcn.h>
#include <sys/stat.h>
#include <utime.h>
#include <unistd.h>

#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <thread>

#include <hip/hiprtc.h>

#include "xg_internal.h"

namespace xg {

uint64_t fnv1a(const std::string& s, uint64_t h) {
  for (unsigned char ch : s) { h ^= ch; h *= 1099511628211ull; }
  return h;
}

std::vector<std::string> base_compile_options(bool strict) {
  return {"--offload-arch=gfx950", "-O3",
          strict ? "-ffp-contract=off" : "-ffp-contract=fast",
          "-fno-gpu-flush-denormals-to-zero",
          // packed fp32 arithmetic is switched off for all generated code
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
}

std::string cache_dir() {
  const char* e = std::getenv("XG_CACHE_DIR");
  std::string d;
  if (e && *e) {
    d = e;
  } else {
    Dl_info info;
    if (dladdr((void*)&cache_dir, &info) && info.dli_fname) {
      std::string f = info.dli_fname;
      size_t k = f.find_last_of('/');
      d = (k == std::string::npos ? std::string(".") : f.substr(0, k)) + "/_kcache";
    } else {
      d = "./_kcache";
    }
  }
  mkdir(d.c_str(), 0775);
  return d;
}

static std::string compiler_tag() {
  int maj = 0, min = 0;
  hiprtcVersion(&maj, &min);
  return "hiprtc" + std::to_string(maj) + "." + std::to_string(min) + "/gfx950/xg1";
}

static bool read_file(const std::string& path, std::vector<char>& buf) {
  std::ifstream f(path, std::ios::binary);
  if (!f) return false;
  f.seekg(0, std::ios::end);
  std::streamoff sz = f.tellg();
  if (sz < 16) return false;
  f.seekg(0);
  buf.resize((size_t)sz);
  f.read(buf.data(), sz);
  if (!f) return false;
  // an AMDGPU code object is an ELF file
  return buf[0] == 0x7f && buf[1] == 'E' && buf[2] == 'L' && buf[3] == 'F';
}

static void write_file_atomic(const std::string& path, const std::vector<char>& buf) {
  std::string tmp = path + ".tmp" + std::to_string(getpid()) + "_" +
                    std::to_string(std::hash<std::thread::id>()(std::this_thread::get_id()));
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return;
  size_t w = std::fwrite(buf.data(), 1, buf.size(), f);
  std::fclose(f);
  if (w == buf.size()) std::rename(tmp.c_str(), path.c_str());
  else std::remove(tmp.c_str());
}

bool compile_hip(const std::string& src, const std::vector<std::string>& opts, CodeObject& co,
                 std::string& err, bool verbose) {
  std::string key = src;
  key.push_back('\0');
  for (auto& o : opts) { key += o; key.push_back('\0'); }
  key += compiler_tag();
  char hex[32];
  std::snprintf(hex, sizeof hex, "%016llx", (unsigned long long)fnv1a(key));
  std::string path = cache_dir() + "/xg-" + hex + ".co";
  if (const char* dd = std::getenv("XG_DUMP_DIR")) {  // keep generated source for inspection
    std::ofstream f(std::string(dd) + "/xg-" + hex + ".hip");
    f << src;
  }
  if (!std::getenv("XG_NO_CACHE") && read_file(path, co.bin)) {
    co.cache_hit = true;
    co.compile_ms = 0;
    (void)utime(path.c_str(), nullptr);  // last use, so stale entries can be pruned by age
    return true;
  }
  auto t0 = std::chrono::steady_clock::now();
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "xg_generated.hip", 0, nullptr, nullptr) !=
      HIPRTC_SUCCESS) {
    err = "hiprtcCreateProgram failed";
    return false;
  }
  std::vector<const char*> o;
  for (auto& s : opts) o.push_back(s.c_str());
  hiprtcResult r = hiprtcCompileProgram(prog, (int)o.size(), o.data());
  if (r != HIPRTC_SUCCESS) {
    size_t ls = 0;
    hiprtcGetProgramLogSize(prog, &ls);
    std::string log(ls, '\0');
    if (ls) hiprtcGetProgramLog(prog, &log[0]);
    err = std::string("hiprtc: ") + hiprtcGetErrorString(r) + "\n" + log.substr(0, 4000);
    hiprtcDestroyProgram(&prog);
    return false;
  }
  size_t cs = 0;
  hiprtcGetCodeSize(prog, &cs);
  co.bin.resize(cs);
  hiprtcGetCode(prog, co.bin.data());
  hiprtcDestroyProgram(&prog);
  auto t1 = std::chrono::steady_clock::now();
  co.compile_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  co.cache_hit = false;
  if (verbose)
    std::fprintf(stderr, "[xg] compiled %zu bytes of source in %.1f ms -> %s\n", src.size(),
                 co.compile_ms, path.c_str());
  write_file_atomic(path, co.bin);
  return true;
}

bool compile_many(const std::vector<std::string>& srcs, const std::vector<std::string>& opts,
                  std::vector<CodeObject>& cos, std::string& err, bool verbose) {
  cos.assign(srcs.size(), CodeObject());
  std::vector<std::string> errs(srcs.size());
  std::vector<char> ok(srcs.size(), 0);
  unsigned hw = std::thread::hardware_concurrency();
  const char* mj = std::getenv("XG_COMPILE_THREADS");
  unsigned nt = mj ? (unsigned)std::atoi(mj) : (hw ? hw : 4);
  if (nt > 16) nt = 16;
  if (nt < 1) nt = 1;
  if (nt > srcs.size()) nt = (unsigned)srcs.size();
  std::atomic<size_t> next{0};
  auto work = [&]() {
    for (size_t i = next++; i < srcs.size(); i = next++)
      ok[i] = compile_hip(srcs[i], opts, cos[i], errs[i], verbose);
  };
  std::vector<std::thread> ts;
  for (unsigned t = 1; t < nt; ++t) ts.emplace_back(work);
  work();
  for (auto& t : ts) t.join();
  for (size_t i = 0; i < srcs.size(); ++i)
    if (!ok[i]) { err = "chunk " + std::to_string(i) + ": " + errs[i]; return false; }
  return true;
}

}  // namespace xg
