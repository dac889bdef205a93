// xg-rtc: compile one generated HIP source for gfx950 with the system ROCm's
// hiprtc and write the code object.  The library runs every compilation in
// one of these helper processes, several at once (hiprtc compilations
// inside one process run one at a time), and always with this hiprtc,
// whatever HIP libraries the calling process has loaded.
//
//   xg-rtc <options file, one option per line> <source file> <output file>
//
// Exit status 0 on success; on failure the compiler log goes to stderr.
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include <unistd.h>

#include <hip/hiprtc.h>

int main(int argc, char** argv) {
  if (argc != 4) {
    std::fprintf(stderr, "usage: xg-rtc <options> <source> <output>\n");
    return 2;
  }
  std::vector<std::string> opts;
  {
    std::ifstream f(argv[1]);
    std::string line;
    while (std::getline(f, line))
      if (!line.empty()) opts.push_back(line);
  }
  std::string src;
  {
    std::ifstream f(argv[2], std::ios::binary);
    if (!f) { std::fprintf(stderr, "xg-rtc: cannot read %s\n", argv[2]); return 2; }
    std::ostringstream ss;
    ss << f.rdbuf();
    src = ss.str();
  }
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "xg_generated.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
    std::fprintf(stderr, "xg-rtc: hiprtcCreateProgram failed\n");
    return 1;
  }
  std::vector<const char*> o;
  for (auto& s : opts) o.push_back(s.c_str());
  hiprtcResult r = hiprtcCompileProgram(prog, (int)o.size(), o.data());
  if (r != HIPRTC_SUCCESS) {
    size_t ls = 0;
    hiprtcGetProgramLogSize(prog, &ls);
    std::string log(ls, '\0');
    if (ls) hiprtcGetProgramLog(prog, &log[0]);
    std::fprintf(stderr, "hiprtc: %s\n%s\n", hiprtcGetErrorString(r), log.substr(0, 4000).c_str());
    hiprtcDestroyProgram(&prog);
    return 1;
  }
  size_t cs = 0;
  hiprtcGetCodeSize(prog, &cs);
  std::vector<char> bin(cs);
  hiprtcGetCode(prog, bin.data());
  hiprtcDestroyProgram(&prog);
  const std::string out = argv[3];
  const std::string tmp = out + ".tmp" + std::to_string(getpid());
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) { std::fprintf(stderr, "xg-rtc: cannot write %s\n", tmp.c_str()); return 1; }
  const size_t w = std::fwrite(bin.data(), 1, bin.size(), f);
  std::fclose(f);
  if (w != bin.size() || std::rename(tmp.c_str(), out.c_str()) != 0) {
    std::remove(tmp.c_str());
    std::fprintf(stderr, "xg-rtc: write failed for %s\n", out.c_str());
    return 1;
  }
  return 0;
}
