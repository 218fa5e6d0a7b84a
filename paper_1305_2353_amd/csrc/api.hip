// C entry points: argument checks, workspace carve-up, kernel launches.

#include <cmath>
#include <cstring>
#include <mutex>

#include "common.h"

namespace ctp {

int launch_compress(int n, int p, const double* a, int lda, int method, double* c, int ldc,
                    int* crow, int* status, void* work, hipStream_t stream);
int launch_pivot_factor(int p, double* a11, int lda, int r, double* R, int ldr, int abs_update,
                        int root, int one_wg, double u, double small, int* perm, int* piv, double* d,
                        int* nelim, int* status, void* state, double* wbuf, hipStream_t stream);
int launch_solve(int n, int p, double* a, int lda, const int* perm, const int* piv, const double* d,
                 const int* nelim, double* w, int ldw, double* lc, int prec, hipStream_t stream);
int launch_schur(int n, int p, const double* a, int lda, const int* piv, const double* d,
                 const int* nelim, int row0, int nrows, double* s, int lds, int tile,
                 hipStream_t stream);
int launch_schur_w(int n, int p, const double* a, int lda, const double* w, int ldw,
                   const int* nelim, int row0, int nrows, double* s, int lds, int variant,
                   hipStream_t stream);
int launch_schur_full(int n, int p, const double* a, int lda, const double* w, int ldw, const int* nelim,
                      double* s, int lds, int tiled, int workgroups, hipStream_t stream);
int launch_form_w(int n, int p, const double* a, int lda, const int* piv, const double* d,
                  const int* nelim, double* w, int ldw, hipStream_t stream);
int launch_lowp_convert(int r, int K, const double* l21, int lda, const double* w, int ldw, const int* nelim,
                        int prec, void* ops, hipStream_t stream);
int launch_lowp_form(int r, int K, const int* nelim, int row0, int nrows, double* s, int lds, int tiled, int prec,
                     void* ops, hipStream_t stream);
size_t lowp_ops_bytes(int r, int kmax);
int launch_tpp_grid(int n, int p, double* a, int lda, int root, double u, double small, int* perm, int* piv,
                    double* d, int* nelim, int* status, double* xt, int* pos, double* part, void* state,
                    double* wbuf, double* xr, int ldr, hipStream_t stream);

size_t batch_header_bytes(int count);
int launch_batch_setup(int count, const ctp_node* in, int method, unsigned flags, double u, double small,
                       double* panels, double* s, int* perm, int* piv, double* d, int* nelim, int* status,
                       void* work, BatchNode** nodes_out, void** pargs_out, unsigned int** counter_out,
                       int reset, hipStream_t stream);
int launch_compress_batch(int count, const BatchNode* nodes, int method, int max_p, int max_r, int max_chunks,
                          hipStream_t stream);
int launch_pivot_batch(int count, const void* pargs, int max_p, int max_r, hipStream_t stream);
int launch_solve_batch(int count, const BatchNode* nodes, int method, int max_p, int max_r, int prec,
                       hipStream_t stream);
int launch_schur_batch(int count, const BatchNode* nodes, int method, long long total, int tiled,
                       int subtract, unsigned int* counter, int variant, int workgroups, hipStream_t stream);

int launch_extend_add(int n, int p, const double* a, int lda, const double* s, int lds, const int* perm,
                      const int* nelim, const int* map, int np, int pp, double* f, int ldf, double* f22,
                      int ld22, int* status, hipStream_t stream);
long long scatter_tiles(int n);
int launch_extend_add_batch(int count, const ctp_scatter_task* tasks, long long tiles, const double* panels,
                            const double* s, const int* perm, const int* nelim, const int* map, double* fpanels,
                            double* f22, int* status, hipStream_t stream);

__global__ void clear_status_kernel(int* status) { *status = 0; }

// Scratch of ctp_supernode_noalloc: one copy per GPU, held until the process
// ends.  Host code never passes the array's name to a kernel (on the host it
// only stands for the symbol): the device address is looked up once per
// device with hipGetSymbolAddress and kept in noalloc_ptr.
static __device__ __align__(256) unsigned char scratch[CTP_NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static void* noalloc_ptr[NOALLOC_MAX_DEVICES];
static std::mutex noalloc_mu;

// Device address of the current device's scratch (looked up on the first
// call on that device, with the device current).
static int noalloc_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return CTP_ERR_HIP_BASE - (int)e;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return CTP_ERR_HIP_BASE - (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(noalloc_mu);
  if (!noalloc_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return CTP_ERR_HIP_BASE - (int)(e != hipSuccess ? e : hipErrorInvalidSymbol);
    noalloc_ptr[dev] = ptr;
  }
  *out = noalloc_ptr[dev];
  return 0;
}

static bool valid_method(int m) { return m >= CTP_TPP && m <= CTP_RESTRICTED; }

// Supernode workspace: the layout of workspace_layout, then (prec FP32 /
// BF16) the reduced-precision operand rows of L21 and W for the Form.
static size_t lowp_region_off(const Workspace& ws) { return align_up(ws.total, 256); }
static size_t supernode_work_bytes(int n, int p, const ctp_opts* o) {
  const Workspace ws = workspace_layout(n, p, o->method);
  if (o->prec == 0 || n <= p || p == 0) return ws.total;
  return lowp_region_off(ws) + lowp_ops_bytes(n - p, p);
}

static int check_opts(const ctp_opts* o) {
  if (!o) return 1;
  if (!valid_method(o->method)) return 1;
  if (!(o->u > 0.0 && o->u <= 0.5)) return 1;
  if (!(o->small >= 0.0) || !std::isfinite(o->small)) return 1;
  if (o->prec < 0 || o->prec > 2) return 1;
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
  *bytes = supernode_work_bytes(n, p, opts);
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

// The Factor task with a host hook that runs once the compression kernels
// (if the rule has any) are enqueued, before the pivot search: the dense
// driver starts the previous panel's deferred trailing update there, so that
// the compression's workgroups do not wait behind that update's.
static int factor_supernode_hooked(int n, int p, double* a, int lda, const ctp_opts* opts, int* perm, int* piv,
                                   double* d, int* nelim, int* status, void* work, size_t lwork,
                                   hipStream_t stream, int (*hook)(void*), void* hook_arg) {
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
  if (hook && (rc = hook(hook_arg)) != 0) return rc;
  const int root = (opts->flags & CTP_FLAG_ROOT) ? 1 : 0;
  const int one_wg = (opts->flags & CTP_FLAG_ONE_WG) ? 1 : 0;
  if (method == CTP_TPP && r > 0 && !one_wg)
    return launch_tpp_grid(n, p, a, lda, root, opts->u, opts->small, perm, piv, d, nelim, status,
                           reinterpret_cast<double*>(base + ws.c_off), reinterpret_cast<int*>(base + ws.j_off),
                           reinterpret_cast<double*>(base + ws.cand_off), base + ws.st_off,
                           reinterpret_cast<double*>(base + ws.wb_off), reinterpret_cast<double*>(base + ws.w_off),
                           ws.ldw, stream);
  return launch_pivot_factor(p, a, lda, rrows, R, ldr, abs_update, root, one_wg, opts->u, opts->small, perm,
                             piv, d, nelim, status, base + ws.st_off,
                             reinterpret_cast<double*>(base + ws.wb_off), stream);
}

int ctp_factor_supernode(int n, int p, double* a, int lda, const ctp_opts* opts, int* perm, int* piv,
                         double* d, int* nelim, int* status, void* work, size_t lwork,
                         hipStream_t stream) {
  return factor_supernode_hooked(n, p, a, lda, opts, perm, piv, d, nelim, status, work, lwork, stream, nullptr,
                                 nullptr);
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
  if (!work || lwork < supernode_work_bytes(n, p, opts)) return -11;
  unsigned char* base = static_cast<unsigned char*>(work);
  double* w = reinterpret_cast<double*>(base + ws.w_off);
  int rc;
  if (opts->method == CTP_TPP) {
    rc = launch_form_w(n, p, a, lda, piv, d, nelim, w, ws.ldw, stream);
  } else {
    double* lc = reinterpret_cast<double*>(base + ws.lc_off);
    rc = launch_solve(n, p, a, lda, perm, piv, d, nelim, w, ws.ldw, lc, opts->prec, stream);
  }
  if (rc || opts->prec == 0 || n <= p || p == 0) return rc;
  // the Form's operand rows in reduced precision
  return launch_lowp_convert(n - p, p, a + p, lda, w, ws.ldw, nelim, opts->prec, base + lowp_region_off(ws), stream);
}

static int supernode_hooked(int n, int p, double* a, int lda, const ctp_opts* opts, int* perm, int* piv,
                            double* d, int* nelim, int* status, double* s, int lds, void* work, size_t lwork,
                            hipStream_t stream, int (*hook)(void*), void* hook_arg) {
  const int r = n - p;
  const bool tiled = opts && (opts->flags & CTP_FLAG_S_TILED);
  if (s && !tiled && lds < (r > 1 ? r : 1)) return -12;
  int rc = factor_supernode_hooked(n, p, a, lda, opts, perm, piv, d, nelim, status, work, lwork, stream, hook,
                                   hook_arg);
  if (rc) return rc == -12 ? -13 : rc;
  rc = ctp_solve_supernode(n, p, a, lda, perm, piv, d, nelim, opts, work, lwork, stream);
  if (rc) return rc == -11 ? -13 : rc;
  if (!s || r <= 0 || p == 0) return 0;
  Workspace ws = workspace_layout(n, p, opts->method);
  if (opts->prec != 0)
    return launch_lowp_form(r, p, nelim, 0, r, s, lds, tiled ? 1 : 0, opts->prec,
                            static_cast<unsigned char*>(work) + lowp_region_off(ws), stream);
  const double* w = reinterpret_cast<const double*>(static_cast<const unsigned char*>(work) + ws.w_off);
  return launch_schur_full(n, p, a, lda, w, ws.ldw, nelim, s, lds, tiled ? 1 : 0, 0, stream);
}

int ctp_supernode(int n, int p, double* a, int lda, const ctp_opts* opts, int* perm, int* piv,
                  double* d, int* nelim, int* status, double* s, int lds, void* work, size_t lwork,
                  hipStream_t stream) {
  return supernode_hooked(n, p, a, lda, opts, perm, piv, d, nelim, status, s, lds, work, lwork, stream, nullptr,
                          nullptr);
}

int ctp_supernode_noalloc(int n, int p, double* a, int lda, const ctp_opts* opts, int* perm, int* piv,
                          double* d, int* nelim, int* status, double* s, int lds, hipStream_t stream) {
  if (n < p) return -1;
  if (p < 0) return -2;
  if (check_opts(opts)) return -5;
  const size_t need = supernode_work_bytes(n, p, opts);
  if (need > CTP_NOALLOC_SCRATCH_BYTES) return CTP_ERR_SCRATCH_TOO_SMALL;
  void* work = nullptr;
  int rc = noalloc_scratch(&work);
  if (rc) return rc;
  return ctp_supernode(n, p, a, lda, opts, perm, piv, d, nelim, status, s, lds, work, CTP_NOALLOC_SCRATCH_BYTES,
                       stream);
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
  if (opts->prec != 0) {
    // reduced precision: the operand rows the Solve converted
    if (!work) return -13;
    if (lwork < supernode_work_bytes(n, p, opts)) return -14;
    if (nrows == 0) return 0;
    const Workspace ws = workspace_layout(n, p, opts->method);
    return launch_lowp_form(n - p, p, nelim, row0, nrows, s, lds, 0, opts->prec,
                            const_cast<unsigned char*>(static_cast<const unsigned char*>(work)) + lowp_region_off(ws),
                            stream);
  }
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



int ctp_batch_plan(int count, ctp_node* nodes, const ctp_opts* opts, ctp_batch_info* info) {
  if (count < 0) return -1;
  if (count > 0 && !nodes) return -2;
  if (check_opts(opts) || opts->method == CTP_TPP) return -3;
  if (!info) return -4;
  ctp_batch_info b;
  std::memset(&b, 0, sizeof(b));
  b.count = count;
  size_t off = batch_header_bytes(count > 0 ? count : 1);
  long long tiles = 0;
  for (int i = 0; i < count; ++i) {
    ctp_node& nd = nodes[i];
    if (nd.p < 1 || nd.p > CTP_MAX_P || nd.n < nd.p || nd.lda < nd.n || nd.a_off < 0 || nd.out_off < 0)
      return -2;
    const int r = nd.n - nd.p;
    if (nd.s_off >= 0 && !(opts->flags & CTP_FLAG_S_TILED) && nd.lds < (r > 1 ? r : 1)) return -2;
    Workspace ws = workspace_layout(nd.n, nd.p, opts->method);
    nd.work_off = (long long)off;
    off = align_up(off + ws.total, 256);
    nd.tile_off = tiles;
    if (nd.s_off >= 0) {
      const long long nt = (r + 127) / 128;
      tiles += nt * (nt + 1) / 2;
    }
    if (nd.p > b.max_p) b.max_p = nd.p;
    if (r > b.max_r) b.max_r = r;
    const int ch = relaxed_chunk_count(r);
    if (ch > b.max_chunks) b.max_chunks = ch;
  }
  b.work_bytes = off;
  b.tiles = tiles;
  *info = b;
  return 0;
}

// The batched calls share one argument check; `need` says which pointers the
// call uses (1: factor outputs, 2: nelim / piv / d read back, 4: S).
static int batch_check(int count, const ctp_node* nodes, const ctp_batch_info* info, double* panels, double* s,
                       int* perm, int* piv, double* d, int* nelim, int* status, const ctp_opts* opts, void* work,
                       size_t lwork, int need) {
  if (count < 0) return -1;
  if (count > 0 && !nodes) return -2;
  if (!info || info->count != count) return -3;
  if (count > 0 && !panels) return -4;
  if (count > 0 && (need & 1) && (!perm || !status)) return -4;
  if (count > 0 && (!piv || !d || !nelim)) return -4;
  if (count > 0 && (need & 4) && !s) return -5;
  if (check_opts(opts) || opts->method == CTP_TPP) return -11;
  if ((opts->flags & CTP_FLAG_S_SUBTRACT) && (opts->flags & CTP_FLAG_S_TILED)) return -11;
  if (!work || lwork < info->work_bytes) return -12;
  return 0;
}

struct BatchLaunch {
  BatchNode* bn = nullptr;
  void* pargs = nullptr;
  unsigned int* counter = nullptr;
};

static int batch_factor(int count, const ctp_node* nodes, const ctp_batch_info* info, double* panels, double* s,
                        int* perm, int* piv, double* d, int* nelim, int* status, const ctp_opts* opts, void* work,
                        BatchLaunch& L, hipStream_t stream) {
  int rc = launch_batch_setup(count, nodes, opts->method, opts->flags, opts->u, opts->small, panels, s, perm, piv,
                              d, nelim, status, work, &L.bn, &L.pargs, &L.counter, 1, stream);
  if (rc) return rc;
  rc = launch_compress_batch(count, L.bn, opts->method, info->max_p, info->max_r, info->max_chunks, stream);
  if (rc) return rc;
  const int rrows = opts->method == CTP_RESTRICTED ? 0 : info->max_p;
  return launch_pivot_batch(count, L.pargs, info->max_p, rrows, stream);
}

static int batch_form(int count, const ctp_batch_info* info, double* s, const ctp_opts* opts, BatchLaunch& L,
                      hipStream_t stream) {
  if (!s || info->tiles <= 0) return 0;
  return launch_schur_batch(count, L.bn, opts->method, info->tiles, (opts->flags & CTP_FLAG_S_TILED) ? 1 : 0,
                            (opts->flags & CTP_FLAG_S_SUBTRACT) ? 1 : 0, L.counter, opts->tile,
                            info->form_workgroups, stream);
}

int ctp_factor_supernode_batched(int count, const ctp_node* nodes, const ctp_batch_info* info, double* panels,
                                 int* perm, int* piv, double* d, int* nelim, int* status, const ctp_opts* opts,
                                 void* work, size_t lwork, hipStream_t stream) {
  int rc = batch_check(count, nodes, info, panels, nullptr, perm, piv, d, nelim, status, opts, work, lwork, 1);
  if (rc || count == 0) return rc;
  BatchLaunch L;
  return batch_factor(count, nodes, info, panels, nullptr, perm, piv, d, nelim, status, opts, work, L, stream);
}

int ctp_solve_supernode_batched(int count, const ctp_node* nodes, const ctp_batch_info* info, double* panels,
                                const int* perm, const int* piv, const double* d, const int* nelim,
                                const ctp_opts* opts, void* work, size_t lwork, hipStream_t stream) {
  int* pm = const_cast<int*>(perm);
  int* pv = const_cast<int*>(piv);
  double* dd = const_cast<double*>(d);
  int* ne = const_cast<int*>(nelim);
  int rc = batch_check(count, nodes, info, panels, nullptr, pm, pv, dd, ne, nullptr, opts, work, lwork, 2);
  if (rc || count == 0) return rc;
  if (!perm) return -5;
  BatchLaunch L;
  // descriptors only: the factorization's outputs stay as they are
  rc = launch_batch_setup(count, nodes, opts->method, opts->flags, opts->u, opts->small, panels, nullptr, pm, pv, dd,
                          ne, ne, work, &L.bn, &L.pargs, &L.counter, 0, stream);
  if (rc) return rc;
  return launch_solve_batch(count, L.bn, opts->method, info->max_p, info->max_r, opts->prec, stream);
}

int ctp_schur_batched(int count, const ctp_node* nodes, const ctp_batch_info* info, const double* panels,
                      const int* piv, const double* d, const int* nelim, double* s, const ctp_opts* opts,
                      void* work, size_t lwork, hipStream_t stream) {
  double* pa = const_cast<double*>(panels);
  int* pv = const_cast<int*>(piv);
  double* dd = const_cast<double*>(d);
  int* ne = const_cast<int*>(nelim);
  int rc = batch_check(count, nodes, info, pa, s, nullptr, pv, dd, ne, nullptr, opts, work, lwork, 2 | 4);
  if (rc || count == 0) return rc;
  BatchLaunch L;
  rc = launch_batch_setup(count, nodes, opts->method, opts->flags, opts->u, opts->small, pa, s, pv, pv, dd, ne, ne,
                          work, &L.bn, &L.pargs, &L.counter, 0, stream);
  if (rc) return rc;
  return batch_form(count, info, s, opts, L, stream);
}

int ctp_supernode_batched(int count, const ctp_node* nodes, const ctp_batch_info* info, double* panels,
                          double* s, int* perm, int* piv, double* d, int* nelim, int* status,
                          const ctp_opts* opts, void* work, size_t lwork, hipStream_t stream) {
  int rc = batch_check(count, nodes, info, panels, nullptr, perm, piv, d, nelim, status, opts, work, lwork, 1);
  if (rc || count == 0) return rc;
  BatchLaunch L;
  rc = batch_factor(count, nodes, info, panels, s, perm, piv, d, nelim, status, opts, work, L, stream);
  if (rc) return rc;
  rc = launch_solve_batch(count, L.bn, opts->method, info->max_p, info->max_r, opts->prec, stream);
  if (rc) return rc;
  return batch_form(count, info, s, opts, L, stream);
}

int ctp_extend_add(int n, int p, const double* a, int lda, const double* s, int lds, const int* perm,
                   const int* nelim, const int* map, int np, int pp, double* f, int ldf, double* f22,
                   int ld22, int* status, hipStream_t stream) {
  if (n < 0) return -1;
  if (p < 0 || p > n) return -2;
  if (!a && p > 0) return -3;
  if (lda < (n > 1 ? n : 1)) return -4;
  if (!s && n > p) return -5;
  if (lds < (n - p > 1 ? n - p : 1)) return -6;
  if (!perm && p > 0) return -7;
  if (!nelim) return -8;
  if (!map && n > 0) return -9;
  if (np < 1) return -10;
  if (pp < 1 || pp > np) return -11;
  if (!f) return -12;
  if (ldf < np) return -13;
  if (!f22 && pp < np) return -14;
  if (pp < np && ld22 < np - pp) return -15;
  return launch_extend_add(n, p, a, lda, s, lds, perm, nelim, map, np, pp, f, ldf, f22, ld22, status, stream);
}

int ctp_scatter_plan(int count, ctp_scatter_task* tasks, long long* tiles) {
  if (count < 0) return -1;
  if (!tasks && count > 0) return -2;
  if (!tiles) return -3;
  long long total = 0;
  for (int k = 0; k < count; ++k) {
    ctp_scatter_task& t = tasks[k];
    const bool ok = t.n >= 1 && t.p >= 0 && t.p <= t.n && t.lda >= t.n && t.node >= 0 && t.a_off >= 0 &&
                    t.out_off >= 0 && t.map_off >= 0 && t.f_off >= 0 && t.np >= 1 && t.pp >= 1 &&
                    t.pp <= t.np && t.ldf >= t.np &&
                    (t.n == t.p || (t.s_off >= 0 && t.lds >= t.n - t.p)) &&
                    (t.pp == t.np || (t.f22_off >= 0 && t.ld22 >= t.np - t.pp));
    if (!ok) return -(100 + k);
    t.tile_off = total;
    total += scatter_tiles(t.n);
  }
  if (total > 0x7fffffffLL) return -4;
  *tiles = total;
  return 0;
}

int ctp_extend_add_batched(int count, const ctp_scatter_task* tasks, long long tiles, const double* panels,
                           const double* s, const int* perm, const int* nelim, const int* map,
                           double* fpanels, double* f22, int* status, hipStream_t stream) {
  if (count < 0) return -1;
  if (count == 0) return 0;
  if (!tasks) return -2;
  if (tiles < 0 || tiles > 0x7fffffffLL) return -3;
  if (!panels || !perm || !nelim || !map || !fpanels) return -4;
  return launch_extend_add_batch(count, tasks, tiles, panels, s, perm, nelim, map, fpanels, f22, status, stream);
}

}  // extern "C"

namespace ctp {
// ctp_supernode with the host hook of factor_supernode_hooked (dense driver).
int supernode_with_hook(int n, int p, double* a, int lda, const ctp_opts* opts, int* perm, int* piv, double* d,
                        int* nelim, int* status, void* work, size_t lwork, hipStream_t stream,
                        int (*hook)(void*), void* hook_arg) {
  return supernode_hooked(n, p, a, lda, opts, perm, piv, d, nelim, status, nullptr, 0, work, lwork, stream, hook,
                          hook_arg);
}
}  // namespace ctp
