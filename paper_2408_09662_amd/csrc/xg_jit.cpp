// Runtime compilation of generated HIP source for gfx950 (hiprtc, run in
// helper processes), with an on-disk code-object cache keyed by a hash of
// source, options and compiler version.  The paper compiles its generated
// file once, offline, with the vendor toolkit; here compilation happens at
// first use and is reused from the cache afterwards, so a program is
// compiled once per machine image.
#include <dlfcn.h>
#include <elf.h>
#include <fcntl.h>
#include <spawn.h>
#include <sys/wait.h>
#include <sys/stat.h>
#include <utime.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <cerrno>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <thread>

#include <unordered_map>

#include <hip/hiprtc.h>

#include "xg_internal.h"

extern char** environ;

namespace xg {

uint64_t fnv1a(const std::string& s, uint64_t h) {
  for (unsigned char ch : s) { h ^= ch; h *= 1099511628211ull; }
  return h;
}

std::vector<std::string> base_compile_options(bool strict) {
  return {"--offload-arch=gfx950", "-O3",
          // outside strict mode the sources permit contraction themselves
          strict ? "-ffp-contract=off" : "-ffp-contract=on",
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

// Cache file of a source under the given options; also keeps the source for
// inspection when XG_DUMP_DIR is set.
static std::string cache_path_of(const std::string& src, const std::vector<std::string>& opts) {
  std::string key = src;
  key.push_back('\0');
  for (auto& o : opts) { key += o; key.push_back('\0'); }
  key += compiler_tag();
  char hex[32];
  std::snprintf(hex, sizeof hex, "%016llx", (unsigned long long)fnv1a(key));
  if (const char* dd = std::getenv("XG_DUMP_DIR")) {
    std::ofstream f(std::string(dd) + "/xg-" + hex + ".hip");
    f << src;
  }
  return cache_dir() + "/xg-" + hex + ".co";
}

static bool cache_hit(const std::string& path, CodeObject& co) {
  if (std::getenv("XG_NO_CACHE") || !read_file(path, co.bin)) return false;
  co.cache_hit = true;
  co.compile_ms = 0;
  (void)utime(path.c_str(), nullptr);  // last use, so stale entries can be pruned by age
  return true;
}

// The helper executable next to this library, or "" if absent.
static std::string helper_path() {
  Dl_info info;
  if (!dladdr((void*)&helper_path, &info) || !info.dli_fname) return "";
  std::string f = info.dli_fname;
  size_t k = f.find_last_of('/');
  std::string h = (k == std::string::npos ? std::string(".") : f.substr(0, k)) + "/xg-rtc";
  return access(h.c_str(), X_OK) == 0 ? h : "";
}

// Compile the sources that miss the cache in helper processes, several at
// once (hiprtc serialises compilations inside one process).  Each helper
// writes its code object to the cache path; false if any failed to start
// or to compile (err then holds the first failure).
static bool compile_in_helpers(const std::vector<std::string>& srcs, const std::vector<size_t>& todo,
                               const std::vector<std::string>& paths, const std::vector<std::string>& opts,
                               const std::string& helper, unsigned procs, std::string& err, bool verbose) {
  const std::string dir = cache_dir();
  // The helpers run with the code-object compiler's own on-disk cache
  // switched off: this library's cache already holds every code object under
  // its source and options, and the other one grows without bound in the
  // user's home directory.
  std::vector<std::string> env_s;
  for (char** e = environ; *e; ++e)
    if (std::strncmp(*e, "AMD_COMGR_CACHE=", 16) != 0) env_s.push_back(*e);
  env_s.push_back("AMD_COMGR_CACHE=0");
  std::vector<char*> envp;
  for (auto& e : env_s) envp.push_back(const_cast<char*>(e.c_str()));
  envp.push_back(nullptr);
  const std::string tag = std::to_string(getpid()) + "_" +
                          std::to_string(std::hash<std::thread::id>()(std::this_thread::get_id()));
  const std::string optf = dir + "/rtc-" + tag + ".opts";
  {
    std::ofstream f(optf);
    for (auto& o : opts) f << o << "\n";
    if (!f) { err = "cannot write " + optf; return false; }
  }
  struct Job { size_t i; pid_t pid; std::string srcf, logf; std::chrono::steady_clock::time_point t0; };
  std::vector<Job> running;
  size_t next = 0;
  bool ok = true;
  // wait for one of this call's own helpers (never for another child of the process)
  auto finish_one = [&]() {
    for (;;) {
      for (size_t r = 0; r < running.size(); ++r) {
        int status = 0;
        const pid_t w = waitpid(running[r].pid, &status, WNOHANG);
        if (w == 0 || (w < 0 && errno == EINTR)) continue;  // still running
        Job j = running[r];
        running.erase(running.begin() + r);
        // w < 0: someone else reaped the child; judge it by its output
        const bool done = w == j.pid ? (WIFEXITED(status) && WEXITSTATUS(status) == 0)
                                      : access(paths[j.i].c_str(), R_OK) == 0;
        if (!done) {
          if (ok) {
            std::ifstream lf(j.logf);
            std::ostringstream ss;
            ss << lf.rdbuf();
            err = "chunk " + std::to_string(j.i) + ": " + ss.str().substr(0, 4000);
          }
          ok = false;
        } else if (verbose) {
          std::fprintf(stderr, "[xg] compiled %zu bytes of source in %.1f ms (helper) -> %s\n",
                       srcs[j.i].size(),
                       std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - j.t0).count(),
                       paths[j.i].c_str());
        }
        std::remove(j.srcf.c_str());
        std::remove(j.logf.c_str());
        return;
      }
      std::this_thread::sleep_for(std::chrono::milliseconds(10));
    }
  };
  while ((next < todo.size() && ok) || !running.empty()) {
    if (next < todo.size() && ok && running.size() < procs) {
      const size_t i = todo[next++];
      Job j;
      j.i = i;
      j.srcf = dir + "/rtc-" + tag + "-" + std::to_string(i) + ".hip";
      j.logf = dir + "/rtc-" + tag + "-" + std::to_string(i) + ".log";
      {
        std::ofstream f(j.srcf, std::ios::binary);
        f << srcs[i];
        if (!f) { err = "cannot write " + j.srcf; ok = false; continue; }
      }
      posix_spawn_file_actions_t fa;
      posix_spawn_file_actions_init(&fa);
      posix_spawn_file_actions_addopen(&fa, 2, j.logf.c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0644);
      posix_spawn_file_actions_addopen(&fa, 1, "/dev/null", O_WRONLY, 0);
      std::vector<std::string> args = {helper, optf, j.srcf, paths[i]};
      std::vector<char*> argv;
      for (auto& a : args) argv.push_back(const_cast<char*>(a.c_str()));
      argv.push_back(nullptr);
      j.t0 = std::chrono::steady_clock::now();
      const int rc = posix_spawn(&j.pid, helper.c_str(), &fa, nullptr, argv.data(), envp.data());
      posix_spawn_file_actions_destroy(&fa);
      if (rc != 0) {
        err = "cannot start " + helper;
        ok = false;
        std::remove(j.srcf.c_str());
        continue;
      }
      running.push_back(j);
      continue;
    }
    finish_one();
  }
  std::remove(optf.c_str());
  return ok;
}

bool compile_many(const std::vector<std::string>& srcs, const std::vector<std::string>& opts,
                  std::vector<CodeObject>& cos, std::string& err, bool verbose) {
  cos.assign(srcs.size(), CodeObject());
  std::vector<std::string> paths(srcs.size());
  std::vector<size_t> todo;
  std::unordered_map<std::string, size_t> first;  // cache path -> first source compiling to it
  for (size_t i = 0; i < srcs.size(); ++i) {
    paths[i] = cache_path_of(srcs[i], opts);
    if (first.count(paths[i])) continue;  // identical source and options: compiled once
    first[paths[i]] = i;
    if (!cache_hit(paths[i], cos[i])) todo.push_back(i);
  }
  auto copy_duplicates = [&]() {
    for (size_t i = 0; i < srcs.size(); ++i) {
      const size_t f = first[paths[i]];
      if (f != i) cos[i] = cos[f];
    }
  };
  if (todo.empty()) { copy_duplicates(); return true; }
  // Misses compile in helper processes, up to XG_COMPILE_PROCS (default:
  // the host's threads, at most 16) at once.  The helper links the system
  // ROCm's hiprtc, so the compiler does not depend on which HIP libraries
  // the calling process happened to load first (a framework may bundle an
  // older copy), and compilations do not share a process.
  const std::string helper = helper_path();
  if (helper.empty()) {
    err = "the compile helper xg-rtc is missing beside libxg.so (build the library again)";
    return false;
  }
  const unsigned hw = std::thread::hardware_concurrency();
  const char* mp = std::getenv("XG_COMPILE_PROCS");
  unsigned procs = mp ? (unsigned)std::max(1, std::atoi(mp)) : (hw ? hw : 4);
  if (procs > 16) procs = 16;
  auto t0 = std::chrono::steady_clock::now();
  if (!compile_in_helpers(srcs, todo, paths, opts, helper, procs, err, verbose)) return false;
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  for (size_t i : todo) {
    if (!read_file(paths[i], cos[i].bin)) {
      err = "the compile helper wrote no code object for chunk " + std::to_string(i);
      return false;
    }
    cos[i].cache_hit = false;
    cos[i].compile_ms = ms / (double)todo.size();
  }
  copy_duplicates();
  return true;
}

bool compile_hip(const std::string& src, const std::vector<std::string>& opts, CodeObject& co,
                 std::string& err, bool verbose) {
  std::vector<CodeObject> cos;
  if (!compile_many({src}, opts, cos, err, verbose)) return false;
  co = std::move(cos[0]);
  return true;
}

namespace {

// The ELF symbol `name` of a code object: file offset of its bytes, or -1.
int64_t symbol_offset(const std::vector<char>& elf, const std::string& name, size_t need) {
  const size_t n = elf.size();
  if (n < sizeof(Elf64_Ehdr)) return -1;
  Elf64_Ehdr eh;
  std::memcpy(&eh, elf.data(), sizeof eh);
  if (std::memcmp(eh.e_ident, ELFMAG, SELFMAG) != 0 || eh.e_ident[EI_CLASS] != ELFCLASS64) return -1;
  if (eh.e_shentsize != sizeof(Elf64_Shdr) || eh.e_shoff == 0 ||
      eh.e_shoff + (uint64_t)eh.e_shnum * sizeof(Elf64_Shdr) > n)
    return -1;
  std::vector<Elf64_Shdr> sh(eh.e_shnum);
  std::memcpy(sh.data(), elf.data() + eh.e_shoff, eh.e_shnum * sizeof(Elf64_Shdr));
  for (const auto& s : sh) {
    if (s.sh_type != SHT_SYMTAB || s.sh_link >= sh.size() || s.sh_entsize != sizeof(Elf64_Sym)) continue;
    const Elf64_Shdr& str = sh[s.sh_link];
    if (s.sh_offset + s.sh_size > n || str.sh_offset + str.sh_size > n) return -1;
    for (uint64_t k = 0; k < s.sh_size / sizeof(Elf64_Sym); ++k) {
      Elf64_Sym sym;
      std::memcpy(&sym, elf.data() + s.sh_offset + k * sizeof(Elf64_Sym), sizeof sym);
      if (sym.st_name >= str.sh_size || sym.st_shndx >= sh.size()) continue;
      const char* nm = elf.data() + str.sh_offset + sym.st_name;
      if (strnlen(nm, str.sh_size - sym.st_name) != name.size() || name != nm) continue;
      const Elf64_Shdr& sec = sh[sym.st_shndx];
      if (sym.st_value < sec.sh_addr) return -1;
      const uint64_t off = sec.sh_offset + (sym.st_value - sec.sh_addr);
      if (off + need > n) return -1;
      return (int64_t)off;
    }
  }
  return -1;
}

// A minimal reader of the MessagePack encoding of the code object's
// metadata note (maps, arrays, strings, integers, booleans, floats, binary).
struct Mp {
  const unsigned char* p;
  const unsigned char* e;
  bool ok = true;
  uint64_t be(int k) {
    if (e - p < k) { ok = false; p = e; return 0; }
    uint64_t v = 0;
    for (int i = 0; i < k; ++i) v = (v << 8) | *p++;
    return v;
  }
  // kinds: 0 nil/bool/float, 1 integer, 2 string, 3 array, 4 map, 5 binary
  struct Tok { int kind = 0; int64_t i = 0; std::string s; uint64_t len = 0; };
  Tok next() {
    Tok t;
    if (p >= e) { ok = false; return t; }
    const unsigned c = *p++;
    if (c <= 0x7f) { t.kind = 1; t.i = c; }
    else if (c >= 0xe0) { t.kind = 1; t.i = (int64_t)(int8_t)c; }
    else if ((c & 0xf0) == 0x80) { t.kind = 4; t.len = c & 0x0f; }
    else if ((c & 0xf0) == 0x90) { t.kind = 3; t.len = c & 0x0f; }
    else if ((c & 0xe0) == 0xa0) { t.kind = 2; t.len = c & 0x1f; }
    else switch (c) {
      case 0xc0: case 0xc2: case 0xc3: break;
      case 0xca: be(4); break;
      case 0xcb: be(8); break;
      case 0xcc: t.kind = 1; t.i = (int64_t)be(1); break;
      case 0xcd: t.kind = 1; t.i = (int64_t)be(2); break;
      case 0xce: t.kind = 1; t.i = (int64_t)be(4); break;
      case 0xcf: t.kind = 1; t.i = (int64_t)be(8); break;
      case 0xd0: t.kind = 1; t.i = (int8_t)be(1); break;
      case 0xd1: t.kind = 1; t.i = (int16_t)be(2); break;
      case 0xd2: t.kind = 1; t.i = (int32_t)be(4); break;
      case 0xd3: t.kind = 1; t.i = (int64_t)be(8); break;
      case 0xd9: t.kind = 2; t.len = be(1); break;
      case 0xda: t.kind = 2; t.len = be(2); break;
      case 0xdb: t.kind = 2; t.len = be(4); break;
      case 0xc4: t.kind = 5; t.len = be(1); break;
      case 0xc5: t.kind = 5; t.len = be(2); break;
      case 0xc6: t.kind = 5; t.len = be(4); break;
      case 0xdc: t.kind = 3; t.len = be(2); break;
      case 0xdd: t.kind = 3; t.len = be(4); break;
      case 0xde: t.kind = 4; t.len = be(2); break;
      case 0xdf: t.kind = 4; t.len = be(4); break;
      default: ok = false; p = e; return t;
    }
    if (t.kind == 2 || t.kind == 5) {
      if ((uint64_t)(e - p) < t.len) { ok = false; p = e; return t; }
      if (t.kind == 2) t.s.assign((const char*)p, (size_t)t.len);
      p += t.len;
    }
    return t;
  }
  void skip(const Tok& t) {  // the contents of an array or map token
    if (t.kind == 3) for (uint64_t i = 0; i < t.len && ok; ++i) skip(next());
    if (t.kind == 4) for (uint64_t i = 0; i < 2 * t.len && ok; ++i) skip(next());
  }
};

// The AMDGPU metadata note's bytes, or an empty range.
std::pair<const unsigned char*, const unsigned char*> metadata_note(const std::vector<char>& elf) {
  const size_t n = elf.size();
  std::pair<const unsigned char*, const unsigned char*> none(nullptr, nullptr);
  if (n < sizeof(Elf64_Ehdr)) return none;
  Elf64_Ehdr eh;
  std::memcpy(&eh, elf.data(), sizeof eh);
  if (eh.e_shentsize != sizeof(Elf64_Shdr) || eh.e_shoff + (uint64_t)eh.e_shnum * sizeof(Elf64_Shdr) > n)
    return none;
  for (int k = 0; k < eh.e_shnum; ++k) {
    Elf64_Shdr s;
    std::memcpy(&s, elf.data() + eh.e_shoff + (uint64_t)k * sizeof s, sizeof s);
    if (s.sh_type != SHT_NOTE || s.sh_offset + s.sh_size > n) continue;
    uint64_t o = s.sh_offset;
    const uint64_t end = s.sh_offset + s.sh_size;
    while (o + 12 <= end) {
      uint32_t nsz, dsz, type;
      std::memcpy(&nsz, elf.data() + o, 4);
      std::memcpy(&dsz, elf.data() + o + 4, 4);
      std::memcpy(&type, elf.data() + o + 8, 4);
      const uint64_t name_o = o + 12, desc_o = name_o + ((nsz + 3) & ~3u);
      if (desc_o + dsz > end) break;
      // NT_AMDGPU_METADATA (32) of owner "AMDGPU"
      if (type == 32 && nsz == 7 && std::memcmp(elf.data() + name_o, "AMDGPU", 6) == 0)
        return {(const unsigned char*)elf.data() + desc_o, (const unsigned char*)elf.data() + desc_o + dsz};
      o = desc_o + ((dsz + 3) & ~3u);
    }
  }
  return none;
}

}  // namespace

bool read_kernel_desc(const std::vector<char>& elf, const std::string& kernel, KernelDesc& kd) {
  // the kernel descriptor "<kernel>.kd" (64 bytes): group segment size at
  // byte 0, private segment size at 4, kernarg size at 8, COMPUTE_PGM_RSRC1
  // at 48, whose bits 5:0 hold the granulated register count (VGPRs +
  // AGPRs of a wave64, granule 8 on gfx950)
  const int64_t off = symbol_offset(elf, kernel + ".kd", 64);
  if (off < 0) return false;
  uint32_t v[13];
  std::memcpy(v, elf.data() + off, sizeof v);
  kd.lds_bytes = v[0];
  kd.scratch_bytes = v[1];
  kd.kernarg_bytes = v[2];
  kd.regs = (int)((v[12] & 0x3f) + 1) * 8;
  return true;
}

int kernel_vgprs(const std::vector<char>& elf, const std::string& kernel) {
  KernelDesc kd;
  return read_kernel_desc(elf, kernel, kd) ? kd.regs : -1;
}

int64_t kernel_hidden_args_offset(const std::vector<char>& elf, const std::string& kernel) {
  // amdhsa.kernels[i] with .name == kernel: the smallest .offset among its
  // .args whose .value_kind starts with "hidden_"
  auto note = metadata_note(elf);
  if (!note.first) return -1;
  Mp m{note.first, note.second};
  Mp::Tok root = m.next();
  if (root.kind != 4) return -1;
  for (uint64_t r = 0; r < root.len && m.ok; ++r) {
    Mp::Tok key = m.next();
    Mp::Tok val = m.next();
    if (!(key.kind == 2 && key.s == "amdhsa.kernels" && val.kind == 3)) { m.skip(val); continue; }
    for (uint64_t k = 0; k < val.len && m.ok; ++k) {
      Mp::Tok kmap = m.next();
      if (kmap.kind != 4) { m.skip(kmap); continue; }
      std::string name;
      int64_t hidden = -1;
      bool have_args = false;
      for (uint64_t f = 0; f < kmap.len && m.ok; ++f) {
        Mp::Tok fk = m.next();
        Mp::Tok fv = m.next();
        if (fk.kind == 2 && fk.s == ".name" && fv.kind == 2) { name = fv.s; continue; }
        if (!(fk.kind == 2 && fk.s == ".args" && fv.kind == 3)) { m.skip(fv); continue; }
        have_args = true;
        for (uint64_t a = 0; a < fv.len && m.ok; ++a) {
          Mp::Tok amap = m.next();
          if (amap.kind != 4) { m.skip(amap); continue; }
          int64_t offset = -1;
          bool is_hidden = false;
          for (uint64_t q = 0; q < amap.len && m.ok; ++q) {
            Mp::Tok ak = m.next();
            Mp::Tok av = m.next();
            if (ak.kind == 2 && ak.s == ".offset" && av.kind == 1) offset = av.i;
            else if (ak.kind == 2 && ak.s == ".value_kind" && av.kind == 2)
              is_hidden = av.s.compare(0, 7, "hidden_") == 0;
            else m.skip(av);
          }
          if (is_hidden && offset >= 0 && (hidden < 0 || offset < hidden)) hidden = offset;
        }
      }
      if (name == kernel && have_args) return hidden;
    }
  }
  return -1;
}

bool check_launch_fits(const std::vector<char>& elf, const std::string& kernel, int block,
                       std::string& err) {
  KernelDesc kd;
  if (!read_kernel_desc(elf, kernel, kd)) { err = "no kernel descriptor for " + kernel + " in its code object"; return false; }
  // a CU has 4 SIMDs with 512 registers per lane each; the waves of one
  // workgroup are spread over the 4 SIMDs and must all be resident at once
  const int per_simd = ((block + 63) / 64 + 3) / 4;
  if (kd.regs * per_simd > 512) {
    err = kernel + " uses " + std::to_string(kd.regs) + " registers per wave: a " + std::to_string(block) +
          "-lane workgroup puts " + std::to_string(per_simd) + " waves on a SIMD, which allows at most " +
          std::to_string(512 / per_simd);
    return false;
  }
  // its LDS (shared variables and spill slots) must fit one CU's 160 KiB
  if (kd.lds_bytes > kLdsBytesPerCU) {
    err = kernel + " needs " + std::to_string(kd.lds_bytes) + " bytes of LDS per workgroup (160 KiB per CU)";
    return false;
  }
  // scratch (registers the compiler spilled to memory) is bounded by the
  // library: the runtime reserves it for every resident lane, and a kernel
  // spilling that much would be far from any useful speed
  if (kd.scratch_bytes > kMaxScratchPerLane) {
    err = kernel + " needs " + std::to_string(kd.scratch_bytes) + " bytes of scratch per lane (at most " +
          std::to_string(kMaxScratchPerLane) + ")";
    return false;
  }
  return true;
}

bool check_kernel_args(const std::vector<char>& elf, const std::string& kernel, int64_t explicit_bytes,
                       std::string& err) {
  const int64_t h = kernel_hidden_args_offset(elf, kernel);
  if (h != ((explicit_bytes + 7) & ~int64_t(7))) {
    err = kernel + ": its implicit arguments start at byte " + std::to_string(h) +
          " of the argument segment, but the code reads its argument block of " +
          std::to_string(explicit_bytes) + " bytes just before them";
    return false;
  }
  return true;
}

}  // namespace xg
