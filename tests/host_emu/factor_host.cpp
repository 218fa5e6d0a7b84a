// Host build of the supernode Factor (compression and pivot search) for the
// sanitizer tests.  TEST INFRASTRUCTURE ONLY.
//
// Links the library's own compress.hip, pivot.hip and tpp.hip, compiled for
// the CPU against the HIP emulation in hip/hip_runtime.h, and runs the same
// sequence of launchers as the library's ctp_factor_supernode entry point:
// compression into C for the compressed rules, then the grid-wide search for
// threshold partial pivoting or the one-workgroup search (decide / apply
// launches, or a single workgroup with CTP_FLAG_ONE_WG) on [A11; R] with
// R = C, A21 or nothing.
//
//   factor_host IN OUT
// IN:  int32 n, p, method, flags; float64 u, small; the n x p panel,
//      column-major (lda = n).
// OUT: the panel after the factorization, then int32 perm[p], piv[p],
//      float64 d[2p], int32 nelim, status, crow[p] (relaxed: the A21 row
//      behind each row of C, -1 for none; other rules: -2).
// The workspace is filled with 0xff bytes (NaN doubles) first, as memory the
// kernels must write before they read.

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "../../paper_1305_2353_amd/csrc/common.h"

namespace ctp {
int launch_compress(int n, int p, const double* a, int lda, int method, double* c, int ldc, int* crow, int* status,
                    void* work, hipStream_t stream);
int launch_pivot_factor(int p, double* a11, int lda, int r, double* R, int ldr, int abs_update, int root,
                        int one_wg, double u, double small, int* perm, int* piv, double* d, int* nelim, int* status,
                        void* state, double* wbuf, hipStream_t stream);
int launch_tpp_grid(int n, int p, double* a, int lda, int root, double u, double small, int* perm, int* piv,
                    double* d, int* nelim, int* status, double* xt, int* pos, double* part, void* state,
                    double* wbuf, double* xr, int ldr, hipStream_t stream);
}  // namespace ctp

using namespace ctp;

static void must(bool ok, const char* what) {
  if (!ok) {
    fprintf(stderr, "factor_host: %s\n", what);
    exit(2);
  }
}

int main(int argc, char** argv) {
  must(argc == 3, "usage: factor_host IN OUT");
  FILE* f = fopen(argv[1], "rb");
  must(f != nullptr, "cannot open input");
  int hdr[4];
  double par[2];
  must(fread(hdr, sizeof(int), 4, f) == 4 && fread(par, sizeof(double), 2, f) == 2, "short header");
  const int n = hdr[0], p = hdr[1], method = hdr[2], flags = hdr[3];
  must(n >= p && p >= 1 && p <= CTP_MAX_P, "bad shape");
  std::vector<double> a((size_t)n * p);
  must(fread(a.data(), sizeof(double), a.size(), f) == a.size(), "short panel");
  fclose(f);

  const int lda = n, r = n - p;
  const Workspace ws = workspace_layout(n, p, method);
  unsigned char* base = static_cast<unsigned char*>(aligned_alloc(256, align_up(ws.total, 256)));
  must(base != nullptr, "workspace allocation");
  memset(base, 0xff, ws.total);
  std::vector<int> perm(p), piv(p);
  std::vector<double> d(2 * (size_t)p);
  int nelim = -1, status = 0;
  const double u = par[0], small = par[1];
  const int root = (flags & CTP_FLAG_ROOT) ? 1 : 0;
  const int one_wg = (flags & CTP_FLAG_ONE_WG) ? 1 : 0;

  int rc = 0;
  double* R = nullptr;
  int ldr = 1, rrows = 0, abs_update = 0;
  if (method == CTP_STRICT || method == CTP_RELAXED) {
    double* c = reinterpret_cast<double*>(base + ws.c_off);
    int* crow = method == CTP_RELAXED ? reinterpret_cast<int*>(base + ws.crow_off) : nullptr;
    rc = launch_compress(n, p, a.data(), lda, method, c, p, crow, &status, base, nullptr);
    R = c;
    ldr = p;
    rrows = p;
    abs_update = method == CTP_STRICT;
  } else if (method == CTP_TPP) {
    R = a.data() + p;
    ldr = lda;
    rrows = r;
  }
  if (rc == 0) {
    if (method == CTP_TPP && r > 0 && !one_wg)
      rc = launch_tpp_grid(n, p, a.data(), lda, root, u, small, perm.data(), piv.data(), d.data(), &nelim, &status,
                           reinterpret_cast<double*>(base + ws.c_off), reinterpret_cast<int*>(base + ws.j_off),
                           reinterpret_cast<double*>(base + ws.cand_off), base + ws.st_off,
                           reinterpret_cast<double*>(base + ws.wb_off), reinterpret_cast<double*>(base + ws.w_off),
                           ws.ldw, nullptr);
    else
      rc = launch_pivot_factor(p, a.data(), lda, rrows, R, ldr, abs_update, root, one_wg, u, small, perm.data(),
                               piv.data(), d.data(), &nelim, &status, base + ws.st_off,
                               reinterpret_cast<double*>(base + ws.wb_off), nullptr);
  }
  must(rc == 0, "a launcher returned an error");
  std::vector<int> crow(p, -2);   // relaxed: the A21 row behind each row of C
  if (method == CTP_RELAXED) memcpy(crow.data(), base + ws.crow_off, sizeof(int) * (size_t)p);
  free(base);

  FILE* o = fopen(argv[2], "wb");
  must(o != nullptr, "cannot open output");
  fwrite(a.data(), sizeof(double), a.size(), o);
  fwrite(perm.data(), sizeof(int), p, o);
  fwrite(piv.data(), sizeof(int), p, o);
  fwrite(d.data(), sizeof(double), 2 * (size_t)p, o);
  fwrite(&nelim, sizeof(int), 1, o);
  fwrite(&status, sizeof(int), 1, o);
  fwrite(crow.data(), sizeof(int), p, o);
  fclose(o);
  return 0;
}
