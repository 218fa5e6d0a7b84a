// C entry points: argument checks, workspace carve-up, kernel launches.

#include <cmath>
#include <cstring>

#include "common.h"

namespace ctp {

int launch_compress(int n, int p, const double* a, int lda, int method, double* c, int ldc,
                    int* crow, int* status, void* work, hipStream_t stream);
int launch_pivot_factor(int p, double* a11, int lda, int r, double* R, int ldr, int abs_update,
                        double u, double small, int* perm, int* piv, double* d, int* nelim,
                        int* status, void* state, double* wbuf, hipStream_t stream);
int launch_solve(int n, int p, double* a, int lda, const int* perm, const int* piv,
                 const double* d, const int* nelim, double* w, int ldw, hipStream_t stream);
int launch_schur(int n, int p, const double* a, int lda, const int* piv, const double* d,
                 const int* nelim, int row0, int nrows, double* s, int lds, int tile,
                 hipStream_t stream);
int launch_schur_w(int n, int p, const double* a, int lda, const double* w, int ldw,
                   const int* nelim, int row0, int nrows, double* s, int lds, int variant,
                   hipStream_t stream);
int launch_form_w(int n, int p, const double* a, int lda, const int* piv, const double* d,
                  const int* nelim, double* w, int ldw, hipStream_t stream);

__global__ void clear_status_kernel(int* status) { *status = 0; }

Workspace workspace_layout(int n, int p, int method) {
  Workspace w;
  const int r = n > p ? n - p : 0;
  size_t off = 0;
  if (method == CTP_STRICT || method == CTP_RELAXED) {
    w.c_off = off;
    off = align_up(off + (size_t)p * p * sizeof(double), 256);
  }
  if (method == CTP_STRICT) {
    w.j_off = off;
    off = align_up(off + (size_t)r * sizeof(int), 256);
  }
  if (method == CTP_RELAXED) {
    w.relaxed_chunks = relaxed_chunk_count(r);
    w.cand_off = off;
    // Cand = {double, int} padded to 16 bytes
    off = align_up(off + (size_t)p * w.relaxed_chunks * RELAXED_TOPK * 16, 256);
    w.crow_off = off;
    off = align_up(off + (size_t)p * sizeof(int), 256);
  }
  w.st_off = off;
  off = align_up(off + (size_t)pivot_state_bytes(), 256);
  w.wb_off = off;
  off = align_up(off + pivot_wbuf_bytes(p), 256);
  if (r > 0) {
    w.ldw = (int)align_up((size_t)r, 32);
    w.w_off = off;
    off = align_up(off + (size_t)w.ldw * p * sizeof(double), 256);
  }
  w.misc_off = off;
  off = align_up(off + 64 * sizeof(int), 256);
  w.total = off;
  return w;
}

static bool valid_method(int m) { return m >= CTP_TPP && m <= CTP_RESTRICTED; }

static int check_opts(const ctp_opts* o) {
  if (!o) return 1;
  if (!valid_method(o->method)) return 1;
  if (!(o->u > 0.0 && o->u <= 0.5)) return 1;
  if (!(o->small >= 0.0) || !std::isfinite(o->small)) return 1;
  return 0;
}

}  // namespace ctp

using namespace ctp;

extern "C" {

void ctp_default_opts(ctp_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->method = CTP_RELAXED;
  o->u = 0.01;
  o->small = 1e-20;
  o->prec = 0;
  o->tile = -1;
  o->flags = 0;
}

const char* ctp_version(void) { return "ctp 0.1 gfx950"; }

int ctp_workspace_size(int n, int p, const ctp_opts* opts, size_t* bytes) {
  if (p < 0) return -2;
  if (n < p) return -1;
  if (check_opts(opts)) return -3;
  if (!bytes) return -4;
  *bytes = workspace_layout(n, p, opts->method).total;
  return 0;
}

int ctp_compress(int n, int p, const double* a, int lda, int method, double* c, int ldc, int* crow,
                 int* status, void* work, size_t lwork, hipStream_t stream) {
  if (n < p) return -1;
  if (p < 0 || p > 2 * CTP_MAX_P) return -2;
  if (!a && n > 0 && p > 0) return -3;
  if (lda < (n > 1 ? n : 1)) return -4;
  if (method != CTP_STRICT && method != CTP_RELAXED) return -5;
  if (!c && p > 0) return -6;
  if (ldc < (p > 1 ? p : 1)) return -7;
  if (!status) return -9;
  Workspace ws = workspace_layout(n, p, method);
  if (!work || lwork < ws.total) return -11;
  if (p == 0) return 0;
  clear_status_kernel<<<1, 1, 0, stream>>>(status);
  return launch_compress(n, p, a, lda, method, c, ldc, crow, status, work, stream);
}

int ctp_factor_supernode(int n, int p, double* a, int lda, const ctp_opts* opts, int* perm, int* piv,
                         double* d, int* nelim, int* status, void* work, size_t lwork,
                         hipStream_t stream) {
  if (n < p) return -1;
  if (p < 0) return -2;
  if (!a && n > 0 && p > 0) return -3;
  if (lda < (n > 1 ? n : 1)) return -4;
  if (check_opts(opts)) return -5;
  if (!perm && p > 0) return -6;
  if (!piv && p > 0) return -7;
  if (!d && p > 0) return -8;
  if (!nelim) return -9;
  if (!status) return -10;
  const int method = opts->method;
  Workspace ws = workspace_layout(n, p, method);
  if (!work || lwork < ws.total) return -12;
  if (p > CTP_MAX_P) return -2;

  clear_status_kernel<<<1, 1, 0, stream>>>(status);
  unsigned char* base = static_cast<unsigned char*>(work);
  const int r = n - p;
  int rc = 0;
  double* R = nullptr;
  int ldr = 1, rrows = 0, abs_update = 0;
  if (method == CTP_STRICT || method == CTP_RELAXED) {
    double* c = reinterpret_cast<double*>(base + ws.c_off);
    int* crow = method == CTP_RELAXED ? reinterpret_cast<int*>(base + ws.crow_off) : nullptr;
    rc = launch_compress(n, p, a, lda, method, c, p, crow, status, work, stream);
    if (rc) return rc;
    R = c;
    ldr = p;
    rrows = p;
    abs_update = method == CTP_STRICT;
  } else if (method == CTP_TPP) {
    R = a + p;
    ldr = lda;
    rrows = r;
  }
  return launch_pivot_factor(p, a, lda, rrows, R, ldr, abs_update, opts->u, opts->small, perm, piv,
                             d, nelim, status, base + ws.st_off,
                             reinterpret_cast<double*>(base + ws.wb_off), stream);
}

int ctp_solve_supernode(int n, int p, double* a, int lda, const int* perm, const int* piv,
                        const double* d, const int* nelim, const ctp_opts* opts, void* work,
                        size_t lwork, hipStream_t stream) {
  if (n < p) return -1;
  if (p < 0 || p > CTP_MAX_P) return -2;
  if (!a && n > 0 && p > 0) return -3;
  if (lda < (n > 1 ? n : 1)) return -4;
  if (!perm && p > 0) return -5;
  if (!piv && p > 0) return -6;
  if (!d && p > 0) return -7;
  if (!nelim) return -8;
  if (check_opts(opts)) return -9;
  Workspace ws = workspace_layout(n, p, opts->method);
  if (!work || lwork < ws.total) return -11;
  double* w = reinterpret_cast<double*>(static_cast<unsigned char*>(work) + ws.w_off);
  if (opts->method == CTP_TPP) return launch_form_w(n, p, a, lda, piv, d, nelim, w, ws.ldw, stream);
  return launch_solve(n, p, a, lda, perm, piv, d, nelim, w, ws.ldw, stream);
}

int ctp_supernode(int n, int p, double* a, int lda, const ctp_opts* opts, int* perm, int* piv,
                  double* d, int* nelim, int* status, void* work, size_t lwork, hipStream_t stream) {
  int rc = ctp_factor_supernode(n, p, a, lda, opts, perm, piv, d, nelim, status, work, lwork, stream);
  if (rc) return rc;
  return ctp_solve_supernode(n, p, a, lda, perm, piv, d, nelim, opts, work, lwork, stream);
}

int ctp_schur(int n, int p, const double* a, int lda, const int* piv, const double* d,
              const int* nelim, int row0, int nrows, double* s, int lds, const ctp_opts* opts,
              const void* work, size_t lwork, hipStream_t stream) {
  if (n < p) return -1;
  if (p < 0 || p > CTP_MAX_P) return -2;
  if (!a && n > 0 && p > 0) return -3;
  if (lda < (n > 1 ? n : 1)) return -4;
  if (!piv && p > 0) return -5;
  if (!d && p > 0) return -6;
  if (!nelim) return -7;
  if (row0 < 0 || row0 > n - p) return -8;
  if (nrows < 0 || row0 + nrows > n - p) return -9;
  if (!s && nrows > 0) return -10;
  if (lds < (nrows > 1 ? nrows : 1)) return -11;
  if (check_opts(opts)) return -12;
  if (work) {
    Workspace ws = workspace_layout(n, p, opts->method);
    if (lwork < ws.total) return -14;
    if (nrows == 0) return 0;
    const double* w =
        reinterpret_cast<const double*>(static_cast<const unsigned char*>(work) + ws.w_off);
    return launch_schur_w(n, p, a, lda, w, ws.ldw, nelim, row0, nrows, s, lds, opts->tile, stream);
  }
  if (nrows == 0) return 0;
  return launch_schur(n, p, a, lda, piv, d, nelim, row0, nrows, s, lds, opts->tile, stream);
}

}  // extern "C"
