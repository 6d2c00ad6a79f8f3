// Build step: writes fast_consts.h, the order-9 (10-point) coefficient table of the tuned 2-D
// kernel as compile-time constants, from the same routine (fill_tab) and the same GLL tables that
// fill the run-time tables, printed as exact hexadecimal floating-point literals.  The kernel
// reads F's and J v's coefficients from these constants: the compiler then forms each one with
// scalar moves next to its use, where the 100 scalar registers of a run-time table would not fit.
#include <cstdio>

#include "fast_common.h"

namespace {
template <int P>
void emit(std::FILE* f) {
  sem::fast::FastTab<double, P> t;
  sem::fast::fill_tab<double, P>(&t);
  auto arr = [&](const char* name, const double* a, int n) {
    std::fprintf(f, "  static constexpr double %s[%d] = {", name, n);
    for (int i = 0; i < n; ++i) std::fprintf(f, "%a%s", a[i], i + 1 < n ? ", " : "");
    std::fprintf(f, "};\n");
  };
  std::fprintf(f, "template <>\nstruct FastConst<%d> {\n", P);
  arr("A", t.A, (P / 2) * (P / 2));
  arr("B", t.B, (P / 2) * (P / 2));
  arr("w", t.w, P);
  arr("imq", t.imq, P);
  arr("D7", t.D7, P);
  arr("Kw", t.Kw, P);
  arr("Dw", t.Dw, P);
  std::fprintf(f, "};\n");
}
}  // namespace

int main(int argc, char** argv) {
  if (argc != 2) {
    std::fprintf(stderr, "usage: %s OUTPUT_HEADER\n", argv[0]);
    return 2;
  }
  std::FILE* f = std::fopen(argv[1], "w");
  if (!f) {
    std::perror(argv[1]);
    return 1;
  }
  std::fprintf(f, "// Generated at build time by gen/fast_consts_gen.hip from fill_tab: do not edit.\n");
  // internal linkage: the compiler folds each coefficient into the code as an immediate; with
  // external linkage it keeps the arrays in memory and loads them like a run-time table
  std::fprintf(f, "#pragma once\n\nnamespace sem {\nnamespace fast {\nnamespace {\n\ntemplate <int P>\nstruct FastConst;\n\n");
  emit<10>(f);
  std::fprintf(f, "\n}  // namespace\n}  // namespace fast\n}  // namespace sem\n");
  return std::fclose(f) == 0 ? 0 : 1;
}
