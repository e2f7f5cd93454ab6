// Host driver for the surrogate's dense linear algebra (gw_linalg.hpp):
// reads a problem from a binary file and writes the result to another.
//   linalg_driver eig  IN OUT   IN: int32 n, then n*n doubles (row-major,
//                               symmetric); OUT: n eigenvalues, then the n*n
//                               eigenvector matrix (eigenvectors as rows)
//   linalg_driver chol IN OUT   IN: int32 n, int32 ncol, n*n doubles (SPD),
//                               n*ncol doubles; OUT: int32 ok, n*ncol doubles
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../paper_2407_19048_amd/csrc/gw_linalg.hpp"

static bool rd(FILE* f, void* p, size_t n) { return std::fread(p, 1, n, f) == n; }
static bool wr(FILE* f, const void* p, size_t n) { return std::fwrite(p, 1, n, f) == n; }

int main(int argc, char** argv) {
  if (argc != 4) return 2;
  FILE* in = std::fopen(argv[2], "rb");
  FILE* out = std::fopen(argv[3], "wb");
  if (!in || !out) return 3;
  int32_t n = 0;
  if (!rd(in, &n, 4) || n < 1) return 4;
  if (std::strcmp(argv[1], "eig") == 0) {
    std::vector<double> a(size_t(n) * n), w;
    if (!rd(in, a.data(), sizeof(double) * a.size())) return 5;
    gw::linalg::sym_eig(a, n, w);
    if (!wr(out, w.data(), sizeof(double) * n) || !wr(out, a.data(), sizeof(double) * a.size())) return 6;
  } else if (std::strcmp(argv[1], "chol") == 0) {
    int32_t ncol = 0;
    if (!rd(in, &ncol, 4) || ncol < 1) return 4;
    std::vector<double> P(size_t(n) * n), rhs(size_t(n) * ncol);
    if (!rd(in, P.data(), sizeof(double) * P.size()) || !rd(in, rhs.data(), sizeof(double) * rhs.size())) return 5;
    const int32_t ok = gw::linalg::chol_solve(P, n, rhs, ncol) ? 1 : 0;
    if (!wr(out, &ok, 4) || !wr(out, rhs.data(), sizeof(double) * rhs.size())) return 6;
  } else {
    return 2;
  }
  std::fclose(in);
  std::fclose(out);
  return 0;
}
