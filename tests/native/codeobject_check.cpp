// Test driver: runs the library's host checks of one kernel of a code
// object file and prints what they read.
//
//   codeobject_check <file.co> <kernel> <block> <explicit argument bytes, or -1>
//
// Prints "regs lds scratch kernarg hidden fits args" (fits, args: 1 or 0)
// and exits 0, or exits 2 if the file cannot be read.
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <iterator>
#include <string>
#include <vector>

#include "xg_internal.h"

int main(int argc, char** argv) {
  if (argc != 5) return 2;
  std::ifstream f(argv[1], std::ios::binary);
  if (!f) return 2;
  std::vector<char> elf((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
  const std::string kernel = argv[2];
  const int block = std::atoi(argv[3]);
  const long long explicit_bytes = std::atoll(argv[4]);
  xg::KernelDesc kd;
  if (!xg::read_kernel_desc(elf, kernel, kd)) return 2;
  std::string err;
  const bool fits = xg::check_launch_fits(elf, kernel, block, err);
  const bool args = explicit_bytes < 0 || xg::check_kernel_args(elf, kernel, explicit_bytes, err);
  std::printf("%d %u %u %u %lld %d %d\n", kd.regs, kd.lds_bytes, kd.scratch_bytes, kd.kernarg_bytes,
              (long long)xg::kernel_hidden_args_offset(elf, kernel), fits ? 1 : 0, args ? 1 : 0);
  if (!err.empty()) std::fprintf(stderr, "%s\n", err.c_str());
  return 0;
}
