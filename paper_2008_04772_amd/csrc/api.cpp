// C ABI of the PMCHWT library (include/pmchwt.h).
//
// Host side: mesh topology and dual-cell tables (geometry.cpp), pair lists,
// quadrature tables, the near-field pattern, and the GMRES control flow
// (Hessenberg matrix and Givens rotations of each right-hand side, a few
// hundred scalars).  Device side: every integral, operator application,
// orthogonalisation and vector update (kernels.hip), and the one-off dense LU
// factorisations of the mass and Gram matrices (rocSOLVER).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <array>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/pmchwt.h"
#include "geometry.hpp"
#include "kernels.hpp"

using namespace pmchwt;
using cd = std::complex<double>;

namespace {

// Device blocks of one context, kept for reuse: a repeated assembly or solve
// of the same problem then allocates and frees nothing (hipFree also waits for
// the whole device).  Blocks are handed out again only within the context,
// whose work is ordered on its stream (side-stream work is joined into it
// before a block returns here), so a reused block is never still in use.
struct BufPool {
  std::multimap<size_t, void*> free;
  size_t cached = 0;
  static constexpr size_t CAP = size_t(96) << 30;  // cached bytes kept at most
  BufPool() = default;
  BufPool(const BufPool&) = delete;
  BufPool& operator=(const BufPool&) = delete;
  ~BufPool() { trim(0); }
  void* take(size_t bytes) {
    auto it = free.find(bytes);
    if (it != free.end()) {
      void* p = it->second;
      free.erase(it);
      cached -= bytes;
      return p;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) == hipSuccess) return p;
    (void)hipGetLastError();
    trim(0);  // give the cached blocks back and try once more
    if (hipMalloc(&p, bytes) == hipSuccess) return p;
    (void)hipGetLastError();
    return nullptr;
  }
  void give(void* p, size_t bytes) {
    free.emplace(bytes, p);
    cached += bytes;
    if (cached > CAP) trim(CAP / 2);
  }
  void trim(size_t keep) {  // largest blocks first
    while (cached > keep && !free.empty()) {
      auto it = std::prev(free.end());
      (void)hipFree(it->second);
      cached -= it->first;
      free.erase(it);
    }
  }
};

struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  BufPool* pool = nullptr;  // owner of the block when it came from a context's pool
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), bytes(o.bytes), pool(o.pool) {
    o.p = nullptr;
    o.bytes = 0;
    o.pool = nullptr;
  }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      pool = o.pool;
      o.p = nullptr;
      o.bytes = 0;
      o.pool = nullptr;
    }
    return *this;
  }
  ~DBuf() { release(); }
  void release() {
    if (p) {
      if (pool)
        pool->give(p, bytes);
      else
        (void)hipFree(p);
    }
    p = nullptr;
    bytes = 0;
    pool = nullptr;
  }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

struct Scat {
  Topo topo;
  DualCells dual;
  bool dual_built = false;
  cd eps, k;
  int edge_off = 0, tri_off = 0, vert_off = 0, cell_off = 0, child_off = 0, bvert_off = 0;
};

struct Fail {
  int code;
  std::string msg;
};

struct CellDev {
  DBuf cell_ptr, ring, child_v, child_vid, child_cen, child_diam2, child_area, coef_ptr, coef, cell_scat;
  DBuf child_cell, child_pos, child_parent, inc_ptr, inc_edges, edge_scat, edge_off;
  int nchild = 0, ncell = 0;
  CellParams params() const {
    CellParams p{};
    p.cell_ptr = cell_ptr.as<int32_t>();
    p.ring = ring.as<int32_t>();
    p.child_v = child_v.as<double>();
    p.child_vid = child_vid.as<int32_t>();
    p.child_cen = child_cen.as<double>();
    p.child_diam2 = child_diam2.as<double>();
    p.child_area = child_area.as<double>();
    p.coef_ptr = coef_ptr.as<int64_t>();
    p.coef = coef.as<double>();
    p.cell_scat = cell_scat.as<int32_t>();
    return p;
  }
};


#define HIPCHK(x)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) throw Fail{PMCHWT_ERR_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)}; \
  } while (0)

}  // namespace

// A BsrMat with the device buffers it points into.
struct BsrHold {
  DBuf bptr, bcol, t1, t2;
  BsrMat m;
  bool valid = false;
};

struct pmchwt_ctx {
  BufPool pool;  // first member: destroyed after every buffer that returns to it
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t side = nullptr;  // look-ahead work of the mass-matrix inverse
  hipEvent_t ev_main = nullptr, ev_side = nullptr;
  rocblas_handle blas = nullptr;
  std::string err;
  double k_ext = 0.0;
  std::vector<Scat> sc;
  int F_tot = 0, E_tot = 0, nv_tot = 0;
  // leading dimensions of the dense operators, padded to a multiple of 16
  // entries: rows start on 128/256-byte boundaries for vector loads, and the
  // real K of the matrix-core product is a multiple of its 32-wide K tile
  int64_t ldE = 0;
  std::vector<int64_t> ldI;
  bool geo_uploaded = false;
  // union geometry (SoA)
  DBuf tv, tcen, tdiam2, tarea, tvid, t2e, tsgn, tscat, edge_off, k_int;
  // A
  bool have_A = false;
  int precA = PMCHWT_FP64;
  DBuf Se, Ce;
  std::vector<DBuf> Si, Ci;
  DBuf Si_ptr, Ci_ptr, ld_int;
  // single scatterer: A^e + A^i pre-combined into three matrices for the GEMV
  // (not for contexts of the serving loop, whose grouped products read the
  // four blocks)
  bool comb = false, comb_ok = true;
  DBuf AC, AS1, AS2;
  // single scatterer, one right-hand side: the same three matrices as upper
  // tiles plus a sparse correction where singular pairs break the symmetry
  // (index tables per geometry, values per assembly); the full combined
  // matrices are then built only when a product with more right-hand sides
  // asks for them
  struct {
    int n = -1, nt = 0;
    int64_t ntiles = 0, nnz = 0;
    DBuf tij, rowptr, crow, col;
    // per correction entry, the singular local-block entries that make it
    // (CSR over the entries; item = block entry << 1 | negate)
    DBuf iptr, item;
    DBuf pack, val, part;
    bool ready = false;
    // the assembly wrote only the upper tiles of Se, Ce, Si, Ci: their lower
    // tiles are filled by mirroring when something first reads them
    bool lower_stale[4] = {false, false, false, false};
  } sym;
  pmchwt_assembly_opts optA{}, optP{};
  // P (near-field BC operators, CSR over union edge indices)
  int precond = -1;
  bool P_int = false, P_ext = false, P_C = false, P_cross = false;
  int64_t nnzP = 0;
  DBuf p_rowptr, p_col, PSi, PCi, PSe, PCe;
  // FP32 copies of the values for the products of a MIXED preconditioner
  // (the FP64 ones stay for copy-out)
  DBuf PSi32, PCi32, PSe32, PCe32;
  // block-sparse copies of the FP32 P (interior per scatterer, exterior)
  std::vector<BsrHold> bsrPi;
  BsrHold bsrPe;
  DBuf soff;  // scatterers' first union edges (device, for the layout kernel)
  int soff_n = -1;
  int64_t soff_E = -1;
  DBuf bsr_ws;  // expanded right-hand blocks of the block-sparse products
  size_t bsr_ws_bytes = 0;
  std::vector<int64_t> h_rowptr;
  std::vector<int32_t> h_col;
  // mass / Gram
  std::vector<DBuf> Minv, MinvT;
  // truncated CSR copies of the FP32 inverses (mixed-precision P): the
  // products for fewer than 16 right-hand sides read these
  struct SparseInv {
    DBuf rowptr, col, val;  // val: float for an FP32 inverse, double for FP64
    int64_t nnz = 0;
    BsrHold bsr;            // block-sparse copy of an FP32 inverse (many right-hand sides)
  };
  std::vector<SparseInv> MinvS, MinvTS;
  // FP64 M_A and M_A^T per scatterer (CSR, scatterer-local indices); when
  // mass_sparse[m], the inverses are the sparse FP32 ones and an FP64
  // preconditioner refines their products against these
  std::vector<SparseInv> MAcsr, MATcsr;
  std::vector<char> mass_sparse;
  // FP64 copy of A (full rows) for the refinement residuals of MIXED solves
  // with many right-hand sides, built on the first such solve after an
  // assembly
  struct {
    bool valid = false;
    DBuf Se, Ce;
    std::vector<DBuf> Si, Ci;
    std::vector<int64_t> ldI;
    int64_t ldE = 0;
  } a64;
  // structural patterns of M_A and M_A^T over the union edges (geometry only)
  struct {
    bool valid = false;
    DBuf rowptr, col, trowptr, tcol;
    std::vector<int64_t> h_rowptr, h_trowptr;
    int maxrow = 0, maxtrow = 0;
  } mp;
  DBuf mass_tmp;  // one vector set of scratch for that refinement
  // RWG Gram matrix (5 nonzeros per row), CSR over union edges with
  // scatterer-local column indices; pattern and slot map built once per geometry
  bool gram_valid = false;
  DBuf g_rowptr, g_col, g_pos, g_val;
  bool mass_f32 = false;  // Minv / MinvT stored in FP32 (preconditioner assembled with MIXED precision)
  // work vectors
  DBuf work;
  size_t work_bytes = 0;
  DBuf mfma_ws;  // expanded right-hand blocks of the matrix-core product
  size_t mfma_ws_bytes = 0;
  pmchwt_profile prof{};
  int64_t count_key = -1, count_pairs = 0, count_pts = 0;
  int64_t calls_A = 0, calls_P = 0;  // operator applications (batched calls) since the last reset
  // index tables that depend only on the meshes (and chi): built once, reused
  // by every assembly of the same geometry (all integrals are recomputed)
  struct {
    bool valid = false;
    double chi = 0;
    bool cross = false;
    DBuf cpairs, slot_off, slot_pos, entry_slots;
    int64_t npairs = 0, bary_pairs = 0, nnz = 0, nslots = 0;
    bool host_valid = false;  // h_rowptr / h_col hold the device pattern
  } nf;
  struct {
    int n = -1;
    DBuf pairs, tab[4];
    int npts[4] = {0, 0, 0, 0};
    int64_t npairs = 0, point_pairs = 0;
    // pairs of each test triangle (the list is sorted by it) and the slot of
    // T+ / T- of every union edge: tables of the matrix-free FP64 product
    DBuf ptr, edge_slots;
    // FP64 local blocks of the singular pairs (the matrix-free FP64 product
    // and the symmetric-tile correction read them)
    DBuf blk;
    // every entry the singular pairs touch and its local-block entries, for
    // the fixed-order scatter into the operators
    DBuf e_row, e_col, e_iptr, e_item;
    int64_t e_nnz = 0;
  } sing;
  DBuf free_slots;  // per-slot sums of the matrix-free FP64 product
  DBuf free_part;   // its regular pairs' partial sums by tile
  bool cells_valid = false;
  CellDev cells;
  std::vector<std::pair<int, int>> slabs;
  size_t slab_elem = 0;
  std::vector<DBuf> slab_rows, slab_rows_l, slab_sp, slab_sm;
  std::vector<int> slab_nrows;
  // trial-edge chunk tables of the atomic-free regular assembly (geometry only)
  int chunk_size = 0, nchunks = 0, max_list = 0;
  DBuf chunk_e, chunk_ptr, chunk_tri, edge_map, edge_scat_d;
  DBuf t1_tmin, ch_tmax;  // tile index bounds of triangles and chunks (upper-tile assembly)
  std::vector<DBuf> slab_cs;  // per slab row: first column of its upper tiles
  double recompute = 0.0;

  // event timings of the solver's operator products, read when the solve ends
  // (or the profile is fetched) instead of waiting on the device per product
  struct PendTime {
    hipEvent_t a, b;
    double* dst;
  };
  std::vector<PendTime> ptimes;
  std::vector<hipEvent_t> evpool;
  int64_t matvec_seq = 0;  // dense products so far (which of them are timed)

  ~pmchwt_ctx() {
    for (auto& p : ptimes) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (auto e : evpool) (void)hipEventDestroy(e);
    if (blas) rocblas_destroy_handle(blas);
    if (ev_main) (void)hipEventDestroy(ev_main);
    if (ev_side) (void)hipEventDestroy(ev_side);
    if (side) (void)hipStreamDestroy(side);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

namespace {

int64_t padld(int64_t n) { return (n + 15) & ~int64_t(15); }

// leading dimension of the inverted mass matrices: a multiple of 32, the K
// tile of the matrix-core product
int64_t ldmass(int64_t n) { return (n + 31) & ~int64_t(31); }

// right-hand sides from which FP32 operators are applied on the matrix cores
constexpr int MFMA_MIN_RHS = 16;
// device bytes of the slot rows of one slab of the regular assembly (pass 1
// output); one slab per scatterer up to this size lets pass 2 overwrite
constexpr double SLAB_BUDGET = 16.0e9;
// automatic choice of the symmetric-tile product: from this many edges on
// (528 tiles of 128 x 128 and up)
constexpr int64_t SYM_MIN_EDGES = 4096;

// ---------------------------------------------------------------------------
// Device scratch of the allocation-free entry point (pmchwt_far_field_noalloc):
// a file-scope array, one copy per GPU, held until the process ends.  Host code
// never passes the array's name to a kernel or a copy (in host code it is a
// host-side stand-in, not a device address); it uses the address that
// hipGetSymbolAddress returned on that device, looked up once per device when
// the first context on it is created.
// ---------------------------------------------------------------------------
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Look up this device's copy of `scratch` (device current); once per device.
hipError_t scratch_setup(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

void* scratch_address(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

double wall_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

template <typename T>
DBuf dalloc(size_t n) {
  DBuf b;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc(&b.p, n * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Fail{PMCHWT_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed"};
  }
  b.bytes = n * sizeof(T);
  return b;
}

// from the context's pool (see BufPool)
template <typename T>
DBuf dalloc_c(pmchwt_ctx* c, size_t n) {
  DBuf b;
  if (n == 0) n = 1;
  b.p = c->pool.take(n * sizeof(T));
  if (!b.p) throw Fail{PMCHWT_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed"};
  b.bytes = n * sizeof(T);
  b.pool = &c->pool;
  return b;
}

// b = a pool block of n elements, the previous one returned first so that a
// same-size block is reused in place
template <typename T>
void realloc_c(pmchwt_ctx* c, DBuf& b, size_t n) {
  b.release();
  b = dalloc_c<T>(c, n);
}

template <typename T>
DBuf upload(pmchwt_ctx* c, const std::vector<T>& v) {
  DBuf b = dalloc_c<T>(c, v.size());
  if (!v.empty()) HIPCHK(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
  return b;
}

int fail(pmchwt_ctx* c, int code, const std::string& m) {
  if (c) c->err = m;
  return code;
}

template <typename F>
int guarded(pmchwt_ctx* c, F&& f) {
  if (!c) return PMCHWT_ERR_INVALID_ARG;
  try {
    HIPCHK(hipSetDevice(c->device));
    int rc = f();
    if (rc == PMCHWT_OK) c->err.clear();
    return rc;
  } catch (const Fail& e) {
    c->err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    c->err = "host allocation failed";
    return PMCHWT_ERR_OUT_OF_MEMORY;
  }
}

// ---------------------------------------------------------------------------
// Quadrature tables (host copies; the kernels read them from constant memory
// or from device tables).
// ---------------------------------------------------------------------------
void triangle_rules(double l[14][3], double w[14]) {
  int k = 0;
  auto orbit = [&](double beta, double wt) {
    const double a = 1.0 - 2.0 * beta;
    const double pts[3][3] = {{a, beta, beta}, {beta, a, beta}, {beta, beta, a}};
    for (int i = 0; i < 3; ++i) {
      for (int d = 0; d < 3; ++d) l[k][d] = pts[i][d];
      w[k++] = wt;
    }
  };
  // degree 1: centroid
  l[k][0] = l[k][1] = l[k][2] = 1.0 / 3.0;
  w[k++] = 1.0;
  // degree 2: orbit (2/3, 1/6, 1/6)
  orbit(1.0 / 6.0, 1.0 / 3.0);
  // degree 3: centroid with weight -27/48 and orbit (3/5, 1/5, 1/5) with 25/48
  l[k][0] = l[k][1] = l[k][2] = 1.0 / 3.0;
  w[k++] = -27.0 / 48.0;
  orbit(0.2, 25.0 / 48.0);
  // degree 4: Dunavant's two-orbit six-point rule
  orbit(0.44594849091596488632, 0.22338158967801146570);
  orbit(0.091576213509770743460, 0.10995174365532186764);
}

void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), pp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p1 = 1.0, p2 = 0.0;
      for (int j = 1; j <= n; ++j) {
        const double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
      }
      pp = n * (z * p1 - p2) / (z * z - 1.0);
      const double z1 = z;
      z = z1 - p1 / pp;
      if (std::fabs(z - z1) < 1e-16) break;
    }
    x[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1.0 - z * z) * pp * pp);
  }
}

// Sauter-Schwab rules on That x That, That = {0 <= x2 <= x1 <= 1}
// (Sauter & Schwab, Boundary Element Methods, Sec. 5.2.1): identical panels
// 6 regions with Jacobian xi^3 eta1^2 eta2, common edge (x2 = 0 shared) 5
// regions (xi^3 eta1^2, then xi^3 eta1^2 eta2), common vertex (origin) 2
// regions with xi^3 eta2.  Records (x1, x2, y1, y2, w).
void sauter_schwab(int kind, int n, std::vector<double>& out) {
  std::vector<double> g, gw;
  gauss_legendre01(n, g, gw);
  out.clear();
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b)
      for (int c = 0; c < n; ++c)
        for (int d = 0; d < n; ++d) {
          const double xi = g[a], e1 = g[b], e2 = g[c], e3 = g[d];
          const double wt = gw[a] * gw[b] * gw[c] * gw[d];
          auto put = [&](double x1, double x2, double y1, double y2, double jac) {
            out.push_back(x1);
            out.push_back(x2);
            out.push_back(y1);
            out.push_back(y2);
            out.push_back(wt * jac);
          };
          if (kind == 3) {
            const double j = xi * xi * xi * e1 * e1 * e2;
            put(xi, xi * (1 - e1 + e1 * e2), xi * (1 - e1 * e2 * e3), xi * (1 - e1), j);
            put(xi * (1 - e1 * e2 * e3), xi * (1 - e1), xi, xi * (1 - e1 + e1 * e2), j);
            put(xi, xi * e1 * (1 - e2 + e2 * e3), xi * (1 - e1 * e2), xi * e1 * (1 - e2), j);
            put(xi * (1 - e1 * e2), xi * e1 * (1 - e2), xi, xi * e1 * (1 - e2 + e2 * e3), j);
            put(xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3), xi, xi * e1 * (1 - e2), j);
            put(xi, xi * e1 * (1 - e2), xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3), j);
          } else if (kind == 2) {
            const double j1 = xi * xi * xi * e1 * e1, j2 = j1 * e2;
            put(xi, xi * e1 * e3, xi * (1 - e1 * e2), xi * e1 * (1 - e2), j1);
            put(xi, xi * e1, xi * (1 - e1 * e2 * e3), xi * e1 * e2 * (1 - e3), j2);
            put(xi * (1 - e1 * e2), xi * e1 * (1 - e2), xi, xi * e1 * e2 * e3, j2);
            put(xi * (1 - e1 * e2 * e3), xi * e1 * e2 * (1 - e3), xi, xi * e1, j2);
            put(xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3), xi, xi * e1 * e2, j2);
          } else {
            const double j = xi * xi * xi * e2;
            put(xi, xi * e1, xi * e2, xi * e2 * e3, j);
            put(xi * e2, xi * e2 * e3, xi, xi * e1, j);
          }
        }
}

struct SSTables {
  DBuf tab[4];
  int npts[4] = {0, 0, 0, 0};
  int n = -1;
};

void build_ss(pmchwt_ctx* c, int n, SSTables& t) {
  for (int kind = 1; kind <= 3; ++kind) {
    std::vector<double> v;
    sauter_schwab(kind, n, v);
    t.npts[kind] = int(v.size() / 5);
    t.tab[kind] = upload(c, v);
  }
  t.n = n;
}

void check_opts(const pmchwt_assembly_opts* o, const char* which) {
  if (!o) throw Fail{PMCHWT_ERR_INVALID_ARG, std::string(which) + " options are NULL"};
  auto okq = [](int q) { return q >= 1 && q <= 4; };
  if (!okq(o->q_near) || !okq(o->q_medium) || !okq(o->q_far))
    throw Fail{PMCHWT_ERR_INVALID_ARG, std::string(which) + ": quadrature orders must be 1..4"};
  if (o->n_singular < 1 || o->n_singular > 8)
    throw Fail{PMCHWT_ERR_INVALID_ARG, std::string(which) + ": n_singular must be 1..8"};
  if (o->precision != PMCHWT_FP64 && o->precision != PMCHWT_MIXED)
    throw Fail{PMCHWT_ERR_INVALID_ARG, std::string(which) + ": unknown precision"};
  if (o->mass_method < 0 || o->mass_method > 2)
    throw Fail{PMCHWT_ERR_INVALID_ARG, std::string(which) + ": mass_method must be 0, 1 or 2"};
  if (o->operator_form < 0 || o->operator_form > 2)
    throw Fail{PMCHWT_ERR_INVALID_ARG, std::string(which) + ": operator_form must be 0, 1 or 2"};
  if (o->mass_hops < 0 || o->mass_hops > 8)
    throw Fail{PMCHWT_ERR_INVALID_ARG, std::string(which) + ": mass_hops must be 0..8"};
}

// ---------------------------------------------------------------------------
// Union geometry upload
// ---------------------------------------------------------------------------
void upload_geometry(pmchwt_ctx* c) {
  if (c->geo_uploaded) return;
  const int F = c->F_tot;
  std::vector<double> tv(9 * size_t(F)), tcen(3 * size_t(F)), tdiam2(F), tarea(F);
  std::vector<int32_t> tvid(3 * size_t(F)), t2e(3 * size_t(F)), tscat(F), eoff, kint_dummy;
  std::vector<int8_t> tsgn(3 * size_t(F));
  for (size_t m = 0; m < c->sc.size(); ++m) {
    const Scat& s = c->sc[m];
    const Topo& T = s.topo;
    for (int f = 0; f < T.F; ++f) {
      const int g = s.tri_off + f;
      double P[3][3];
      for (int k = 0; k < 3; ++k)
        for (int d = 0; d < 3; ++d) {
          P[k][d] = T.v[3 * size_t(T.t[3 * f + k]) + d];
          tv[size_t(3 * k + d) * F + g] = P[k][d];
        }
      for (int d = 0; d < 3; ++d) tcen[size_t(d) * F + g] = (P[0][d] + P[1][d] + P[2][d]) / 3.0;
      double dm = 0.0;
      const int pr[3][2] = {{0, 1}, {1, 2}, {2, 0}};
      for (auto& q : pr) {
        const double ex = P[q[0]][0] - P[q[1]][0], ey = P[q[0]][1] - P[q[1]][1], ez = P[q[0]][2] - P[q[1]][2];
        const double e2 = ex * ex + ey * ey + ez * ez;
        dm = std::max(dm, e2);
      }
      tdiam2[g] = dm;
      tarea[g] = T.area[f];
      for (int a = 0; a < 3; ++a) {
        tvid[size_t(a) * F + g] = s.vert_off + T.t[3 * f + a];
        t2e[size_t(a) * F + g] = s.edge_off + T.t2e[3 * f + a];
        tsgn[size_t(a) * F + g] = T.sgn[3 * f + a];
      }
      tscat[g] = int32_t(m);
    }
    eoff.push_back(s.edge_off);
  }
  c->tv = upload(c, tv);
  c->tcen = upload(c, tcen);
  c->tdiam2 = upload(c, tdiam2);
  c->tarea = upload(c, tarea);
  c->tvid = upload(c, tvid);
  c->t2e = upload(c, t2e);
  c->tsgn = upload(c, tsgn);
  c->tscat = upload(c, tscat);
  c->edge_off = upload(c, eoff);
  c->geo_uploaded = true;
}

void upload_k(pmchwt_ctx* c) {
  std::vector<double> k;
  for (auto& s : c->sc) {
    s.k = c->k_ext * std::sqrt(s.eps);
    k.push_back(s.k.real());
    k.push_back(s.k.imag());
  }
  c->k_int = upload(c, k);
}

template <typename M>
AsmParams<M> asm_params(pmchwt_ctx* c) {
  AsmParams<M> p{};
  p.F = c->F_tot;
  p.tv = c->tv.as<double>();
  p.tcen = c->tcen.as<double>();
  p.tdiam2 = c->tdiam2.as<double>();
  p.tarea = c->tarea.as<double>();
  p.tvid = c->tvid.as<int32_t>();
  p.t2e = c->t2e.as<int32_t>();
  p.tsgn = c->tsgn.as<int8_t>();
  p.tscat = c->tscat.as<int32_t>();
  p.edge_off = c->edge_off.as<int32_t>();
  p.k_int = c->k_int.as<double>();
  p.k_ext = c->k_ext;
  p.Se = c->Se.as<M>();
  p.Ce = c->Ce.as<M>();
  p.ld_ext = c->ldE;
  p.Si = c->Si_ptr.as<M*>();
  p.Ci = c->Ci_ptr.as<M*>();
  p.ld_int = c->ld_int.as<int64_t>();
  return p;
}

// Fill the lower tiles of the operators in `mask` (1 Se, 2 Ce, 4 Si, 8 Ci)
// that an upper-tile assembly left stale (one scatterer): the mirror of the
// upper tiles plus the singular pairs' asymmetry on the correction entries.
void ensure_lower(pmchwt_ctx* c, int mask) {
  const int n = c->E_tot;
  for (int op = 0; op < 4; ++op) {
    if (!(mask & (1 << op)) || !c->sym.lower_stale[op]) continue;
    DBuf& X = op == 0 ? c->Se : (op == 1 ? c->Ce : (op == 2 ? c->Si[0] : c->Ci[0]));
    const int64_t ld = op < 2 ? c->ldE : c->ldI[0];
    if (c->precA == PMCHWT_FP64)
      launch_mirror_lower<double>(X.as<double>(), ld, n, c->sym.crow.as<int32_t>(), c->sym.col.as<int32_t>(),
                                  c->sym.iptr.as<int64_t>(), c->sym.item.as<int32_t>(), c->sing.blk.as<double>(),
                                  c->sym.nnz, op, c->stream);
    else
      launch_mirror_lower<float>(X.as<float>(), ld, n, c->sym.crow.as<int32_t>(), c->sym.col.as<int32_t>(),
                                 c->sym.iptr.as<int64_t>(), c->sym.item.as<int32_t>(), c->sing.blk.as<double>(),
                                 c->sym.nnz, op, c->stream);
    HIPCHK(hipGetLastError());
    c->sym.lower_stale[op] = false;
  }
}

void flush_times(pmchwt_ctx* c);

// Timer whose result is added to *dst later (flush_times): no host wait.
struct LazyTimer {
  pmchwt_ctx* c;
  hipEvent_t a = nullptr;
  static hipEvent_t take(pmchwt_ctx* c) {
    if (!c->evpool.empty()) {
      hipEvent_t e = c->evpool.back();
      c->evpool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    HIPCHK(hipEventCreate(&e));
    return e;
  }
  explicit LazyTimer(pmchwt_ctx* c_, bool on = true) : c(c_) {
    if (!on) return;
    a = take(c);
    HIPCHK(hipEventRecord(a, c->stream));
  }
  void stop(double* dst) {
    if (!a) return;
    hipEvent_t b = take(c);
    c->ptimes.push_back({a, b, dst});
    a = nullptr;
    HIPCHK(hipEventRecord(b, c->stream));
    if (c->ptimes.size() >= 4096) flush_times(c);  // bounded between solves too
  }
  ~LazyTimer() {
    if (a) c->evpool.push_back(a);
  }
};

// Dense products timed: one in MATVEC_SAMPLE (a pair of timing events
// between two kernels costs a few microseconds of idle device time)
constexpr int MATVEC_SAMPLE = 8;
bool sample_matvec(pmchwt_ctx* c) { return c->matvec_seq++ % MATVEC_SAMPLE == 0; }

// add the pending timings to their counters (waits for their events)
void flush_times(pmchwt_ctx* c) {
  for (auto& p : c->ptimes) {
    HIPCHK(hipEventSynchronize(p.b));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
    *p.dst += ms;
    c->evpool.push_back(p.a);
    c->evpool.push_back(p.b);
  }
  c->ptimes.clear();
}

struct EvTimer {
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t s;
  explicit EvTimer(hipStream_t st) : s(st) {
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    HIPCHK(hipEventRecord(a, s));
  }
  double stop() {
    HIPCHK(hipEventRecord(b, s));
    HIPCHK(hipEventSynchronize(b));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, a, b));
    return ms;
  }
  ~EvTimer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// ---------------------------------------------------------------------------
// Assembly of A
// ---------------------------------------------------------------------------
// the full combined matrices C, S1, S2 of a single scatterer
template <typename M>
void build_comb(pmchwt_ctx* c) {
  ensure_lower(c, 15);
  const Scat& s = c->sc[0];
  const int64_t ne = c->E_tot * c->ldE;
  realloc_c<M>(c, c->AC, size_t(2 * ne));
  realloc_c<M>(c, c->AS1, size_t(2 * ne));
  realloc_c<M>(c, c->AS2, size_t(2 * ne));
  launch_combine3<M>(c->Se.as<M>(), c->Ce.as<M>(), c->Si[0].as<M>(), c->Ci[0].as<M>(), ne, c->k_ext, s.k.real(),
                     s.k.imag(), c->AC.as<M>(), c->AS1.as<M>(), c->AS2.as<M>(), c->stream);
  HIPCHK(hipGetLastError());
  c->comb = true;
}

// Copies of a few device scalars to the host (one synchronisation).
void read_scalars(pmchwt_ctx* c, std::initializer_list<std::pair<void*, std::pair<const void*, size_t>>> items) {
  for (auto& it : items) HIPCHK(hipMemcpyAsync(it.first, it.second.first, it.second.second, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
}

int pow2_ceil(int64_t n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// Records (row, column, singular local-block entry) grouped per entry:
// crow / col of each entry in row-major order, iptr its first record (with
// iptr[nnz] = the record count) and item the records in (column, item)
// order.  all = 0: the correction entries below the diagonal tiles of the
// symmetric-tile storage; all = 1: every entry a singular pair touches.
struct RecTables {
  DBuf rowptr, crow, col, iptr, item;
  int64_t nnz = 0;
};

RecTables rec_tables(pmchwt_ctx* c, bool all) {
  const int n = int(c->E_tot);
  hipStream_t st = c->stream;
  if (9 * c->sing.npairs >= (int64_t(1) << 30))
    throw Fail{PMCHWT_ERR_INVALID_MESH, "too many singular pairs for the 31-bit record items"};
  SymRecJob J{};
  J.npairs = c->sing.npairs;
  J.pairs = c->sing.pairs.as<int32_t>();
  J.t2e = c->t2e.as<int32_t>();
  J.F = c->F_tot;
  J.tile = SYM_T;
  J.n = n;
  J.all = all ? 1 : 0;
  DBuf cnt = dalloc_c<int32_t>(c, size_t(n)), stats = dalloc_c<int32_t>(c, 4);
  DBuf recptr = dalloc_c<int64_t>(c, size_t(n) + 1);
  RecTables o;
  o.rowptr = dalloc_c<int64_t>(c, size_t(n) + 1);
  launch_cls_fill_i32(cnt.as<int32_t>(), n, 0, st);
  launch_cls_fill_i32(stats.as<int32_t>(), 4, 0, st);
  J.cnt = cnt.as<int32_t>();
  J.maxrec = stats.as<int32_t>();
  launch_sym_records(J, 0, st);
  launch_scan_i32(cnt.as<int32_t>(), n, recptr.as<int64_t>(), st);
  HIPCHK(hipGetLastError());
  int64_t nrec = 0;
  int32_t maxrec = 0;
  read_scalars(c, {{&nrec, {recptr.as<int64_t>() + n, 8}}, {&maxrec, {stats.as<int32_t>(), 4}}});
  if (maxrec > 4096) throw Fail{PMCHWT_ERR_INVALID_MESH, "vertex valence too high for the singular-entry tables"};
  DBuf rec = dalloc_c<int64_t>(c, size_t(std::max<int64_t>(nrec, 1)));
  launch_cls_fill_i32(cnt.as<int32_t>(), n, 0, st);
  J.recptr = recptr.as<int64_t>();
  J.cur = cnt.as<int32_t>();
  J.rec = rec.as<int64_t>();
  launch_sym_records(J, 1, st);
  launch_sym_sort(J, pow2_ceil(std::max(maxrec, 1)), st);
  launch_scan_i32(cnt.as<int32_t>(), n, o.rowptr.as<int64_t>(), st);
  HIPCHK(hipGetLastError());
  read_scalars(c, {{&o.nnz, {o.rowptr.as<int64_t>() + n, 8}}});
  o.crow = dalloc_c<int32_t>(c, size_t(std::max<int64_t>(o.nnz, 1)));
  o.col = dalloc_c<int32_t>(c, size_t(std::max<int64_t>(o.nnz, 1)));
  o.iptr = dalloc_c<int64_t>(c, size_t(o.nnz) + 1);
  o.item = dalloc_c<int32_t>(c, size_t(std::max<int64_t>(nrec, 1)));
  J.rowptr = o.rowptr.as<int64_t>();
  J.crow = o.crow.as<int32_t>();
  J.col = o.col.as<int32_t>();
  J.iptr = o.iptr.as<int64_t>();
  J.item = o.item.as<int32_t>();
  launch_sym_emit(J, st);
  launch_cls_set_i64(o.iptr.as<int64_t>() + o.nnz, nrec, st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));  // the scratch tables above go out of scope
  return o;
}

// Index tables of the symmetric-tile form (one scatterer, geometry only):
// the upper tiles in row-major order (host) and the correction pattern, i.e.
// every entry (r, c) below the diagonal tiles that a pair of triangles
// sharing a vertex (the Sauter-Schwab pairs) contributes to, with the
// singular local-block entries that make it: + for those added to X_rc, -
// for those added to X_cr (classification kernels, from the device pair list).
void sym_tables(pmchwt_ctx* c) {
  const int n = int(c->E_tot);
  if (c->sym.n == n) return;
  const int nt = (n + SYM_T - 1) / SYM_T;
  std::vector<int32_t> tij;
  for (int I = 0; I < nt; ++I)
    for (int J = I; J < nt; ++J) {
      tij.push_back(I);
      tij.push_back(J);
    }
  RecTables r = rec_tables(c, false);
  c->sym.crow = std::move(r.crow);
  c->sym.col = std::move(r.col);
  c->sym.iptr = std::move(r.iptr);
  c->sym.item = std::move(r.item);
  c->sym.rowptr = std::move(r.rowptr);
  c->sym.nt = nt;
  c->sym.ntiles = int64_t(tij.size() / 2);
  c->sym.nnz = r.nnz;
  c->sym.tij = upload(c, tij);
  c->sym.n = n;
  HIPCHK(hipStreamSynchronize(c->stream));
}

// Singular pairs (ordered triangle pairs sharing at least one vertex; the
// pairs of a test triangle contiguous, trial triangles ascending) and their
// Sauter-Schwab point pairs, by the classification kernels.  The host only
// lists the triangles at each vertex (counting sort, O(F)).
void singular_list(pmchwt_ctx* c, const int* npts) {
  hipStream_t st = c->stream;
  const int F = c->F_tot;
  std::vector<int32_t> vptr(size_t(c->nv_tot) + 1, 0), v2t(3 * size_t(F));
  for (auto& s : c->sc)
    for (int f = 0; f < s.topo.F; ++f)
      for (int a = 0; a < 3; ++a) ++vptr[size_t(s.vert_off + s.topo.t[3 * size_t(f) + a]) + 1];
  for (size_t v = 0; v + 1 < vptr.size(); ++v) vptr[v + 1] += vptr[v];
  {
    std::vector<int32_t> cur(vptr.begin(), vptr.end() - 1);
    for (auto& s : c->sc)
      for (int f = 0; f < s.topo.F; ++f)
        for (int a = 0; a < 3; ++a) v2t[size_t(cur[size_t(s.vert_off + s.topo.t[3 * size_t(f) + a])]++)] = s.tri_off + f;
  }
  DBuf d_vptr = upload(c, vptr), d_v2t = upload(c, v2t);
  DBuf cnt = dalloc_c<int32_t>(c, size_t(F)), stats = dalloc_c<int32_t>(c, 4), pts = dalloc_c<int64_t>(c, 1);
  DBuf sptr = dalloc_c<int64_t>(c, size_t(F) + 1);
  launch_cls_fill_i32(stats.as<int32_t>(), 4, 0, st);
  launch_cls_set_i64(pts.as<int64_t>(), 0, st);
  SingListJob J{};
  J.F = F;
  J.tvid = c->tvid.as<int32_t>();
  J.v2t_ptr = d_vptr.as<int32_t>();
  J.v2t = d_v2t.as<int32_t>();
  J.cnt = cnt.as<int32_t>();
  J.flag = stats.as<int32_t>();
  for (int k = 0; k < 4; ++k) J.npts[k] = npts[k];
  launch_sing_list(J, false, st);
  launch_scan_i32(cnt.as<int32_t>(), F, sptr.as<int64_t>(), st);
  HIPCHK(hipGetLastError());
  int64_t npairs = 0;
  int32_t over = 0;
  read_scalars(c, {{&npairs, {sptr.as<int64_t>() + F, 8}}, {&over, {stats.as<int32_t>(), 4}}});
  if (over)
    throw Fail{PMCHWT_ERR_INVALID_MESH, "a triangle shares a vertex with more than " +
                                            std::to_string(sing_neighbour_capacity()) + " triangles"};
  c->sing.pairs = dalloc_c<int32_t>(c, size_t(2 * std::max<int64_t>(npairs, 1)));
  J.sptr = sptr.as<int64_t>();
  J.pairs = c->sing.pairs.as<int32_t>();
  J.point_pairs = reinterpret_cast<unsigned long long*>(pts.p);
  launch_sing_list(J, true, st);
  HIPCHK(hipGetLastError());
  int64_t np = 0;
  read_scalars(c, {{&np, {pts.p, 8}}});
  c->sing.ptr = std::move(sptr);
  c->sing.npairs = npairs;
  c->sing.point_pairs = np;
}

template <typename M>
void assemble_A_impl(pmchwt_ctx* c, const pmchwt_assembly_opts& o) {
  const int64_t E = c->E_tot;
  c->ldE = padld(E);
  realloc_c<M>(c, c->Se, size_t(2 * E * c->ldE));
  realloc_c<M>(c, c->Ce, size_t(2 * E * c->ldE));
  std::vector<M*> sp, cp;
  std::vector<int64_t> lds;
  c->Si.clear();
  c->Ci.clear();
  c->ldI.clear();
  for (auto& s : c->sc) {
    const int64_t Em = s.topo.E, ld = padld(Em);
    c->Si.push_back(dalloc_c<M>(c, size_t(2 * Em * ld)));
    c->Ci.push_back(dalloc_c<M>(c, size_t(2 * Em * ld)));
    sp.push_back(c->Si.back().as<M>());
    cp.push_back(c->Ci.back().as<M>());
    lds.push_back(ld);
    c->ldI.push_back(ld);
  }
  c->Si_ptr = upload(c, sp);
  c->Ci_ptr = upload(c, cp);
  c->ld_int = upload(c, lds);
  auto zero = [&](DBuf& b) {
    if (sizeof(M) == 8)
      launch_zero(reinterpret_cast<double*>(b.p), int64_t(b.bytes / 8), c->stream);
    else
      launch_zero_f(reinterpret_cast<float*>(b.p), int64_t(b.bytes / 4), c->stream);
  };
  AsmParams<M> p = asm_params<M>(c);
  p.q_near = o.q_near;
  p.q_medium = o.q_medium;
  p.q_far = o.q_far;

  // singular pair list (ordered pairs sharing at least one vertex) and the
  // Sauter-Schwab tables of order n: index tables, built once per geometry
  if (c->sing.n != o.n_singular) {
    const double wt = wall_ms();
    SSTables ss;
    build_ss(c, o.n_singular, ss);
    const int npts_by_shared[4] = {0, ss.npts[1], ss.npts[2], ss.npts[3]};
    singular_list(c, npts_by_shared);
    {
      RecTables r = rec_tables(c, true);
      c->sing.e_row = std::move(r.crow);
      c->sing.e_col = std::move(r.col);
      c->sing.e_iptr = std::move(r.iptr);
      c->sing.e_item = std::move(r.item);
      c->sing.e_nnz = r.nnz;
    }
    std::vector<int32_t> eslot(2 * size_t(c->E_tot), 0);
    for (auto& sc : c->sc)
      for (int f = 0; f < sc.topo.F; ++f)
        for (int a = 0; a < 3; ++a) {
          const int e = sc.edge_off + sc.topo.t2e[3 * f + a];
          eslot[2 * size_t(e) + (sc.topo.sgn[3 * f + a] > 0 ? 0 : 1)] = 3 * (sc.tri_off + f) + a;
        }
    c->sing.edge_slots = upload(c, eslot);
    for (int k = 1; k <= 3; ++k) {
      c->sing.tab[k] = std::move(ss.tab[k]);
      c->sing.npts[k] = ss.npts[k];
    }
    c->sing.n = o.n_singular;
    c->prof.wall_tables_A += wall_ms() - wt;
  }
  SingParams sp_{};
  sp_.npairs = c->sing.npairs;
  sp_.pairs = c->sing.pairs.as<int32_t>();
  for (int k = 1; k <= 3; ++k) {
    sp_.tab[k] = c->sing.tab[k].as<double>();
    sp_.npts[k] = c->sing.npts[k];
  }
  const int64_t npts_sing = c->sing.point_pairs;
  // trial-edge chunks: runs of consecutive edges whose distinct T+/T-
  // triangles number at most the regular kernel's workgroup size (256 in
  // FP32, 128 in FP64, where the moments take twice the LDS)
  const int CH = regular_chunk_limit(sizeof(M) == 8);
  if (c->chunk_size != CH) {
    const double wt = wall_ms();
    std::vector<int32_t> tp(c->E_tot), tm(c->E_tot), escat(c->E_tot);
    std::vector<int8_t> bp(c->E_tot), bm(c->E_tot);
    for (size_t m = 0; m < c->sc.size(); ++m) {
      const Scat& s = c->sc[m];
      for (int f = 0; f < s.topo.F; ++f)
        for (int a = 0; a < 3; ++a) {
          const int e = s.edge_off + s.topo.t2e[3 * f + a];
          if (s.topo.sgn[3 * f + a] > 0) {
            tp[e] = s.tri_off + f;
            bp[e] = int8_t(a);
          } else {
            tm[e] = s.tri_off + f;
            bm[e] = int8_t(a);
          }
        }
      for (int e = 0; e < s.topo.E; ++e) escat[s.edge_off + e] = int32_t(m);
    }
    std::vector<int32_t> cptr{0}, ctri, cedge{0};
    std::vector<int16_t> emap(4 * size_t(c->E_tot));
    // chunk membership of each trial triangle by stamp (the chunk index)
    std::vector<int32_t> stamp(size_t(c->F_tot), -1);
    std::vector<int16_t> spos(size_t(c->F_tot), 0);
    int chunk = 0, held = 0, maxl = 0;
    auto slot = [&](int32_t t) -> int16_t {
      if (stamp[t] != chunk) {
        stamp[t] = chunk;
        spos[t] = int16_t(held++);
        ctri.push_back(t);
      }
      return spos[t];
    };
    for (int j = 0; j < c->E_tot; ++j) {
      const int add = int(stamp[tp[j]] != chunk) + int(stamp[tm[j]] != chunk);
      if (held + add > CH) {  // close the chunk before edge j
        maxl = std::max(maxl, held);
        cptr.push_back(int32_t(ctri.size()));
        cedge.push_back(j);
        ++chunk;
        held = 0;
      }
      emap[4 * size_t(j) + 0] = slot(tp[j]);
      emap[4 * size_t(j) + 1] = bp[j];
      emap[4 * size_t(j) + 2] = slot(tm[j]);
      emap[4 * size_t(j) + 3] = bm[j];
    }
    maxl = std::max(maxl, held);
    cptr.push_back(int32_t(ctri.size()));
    cedge.push_back(c->E_tot);
    const int nch = int(cedge.size()) - 1;
    c->chunk_e = upload(c, cedge);
    c->chunk_ptr = upload(c, cptr);
    c->chunk_tri = upload(c, ctri);
    c->edge_map = upload(c, emap);
    c->edge_scat_d = upload(c, escat);
    c->nchunks = nch;
    c->max_list = maxl;
    c->recompute = double(ctri.size()) / double(c->F_tot);
    c->chunk_size = CH;
    std::vector<int32_t> tmin(c->F_tot), tmax(nch);
    for (auto& sc : c->sc)
      for (int f = 0; f < sc.topo.F; ++f) {
        int m = INT32_MAX;
        for (int a = 0; a < 3; ++a) m = std::min(m, (sc.edge_off + sc.topo.t2e[3 * f + a]) / SYM_T);
        tmin[sc.tri_off + f] = m;
      }
    for (int ch = 0; ch < nch; ++ch) tmax[ch] = (cedge[ch + 1] - 1) / SYM_T;
    c->t1_tmin = upload(c, tmin);
    c->ch_tmax = upload(c, tmax);
    c->prof.wall_tables_A += wall_ms() - wt;
  }
  // one scatterer stored as symmetric tiles: only the upper tiles are
  // assembled (the lower ones are their mirror, filled on first use)
  const int form = c->optA.operator_form;
  const bool symform = c->sc.size() == 1 && c->comb_ok && (form == 2 || (form == 0 && E >= SYM_MIN_EDGES));
  // slabs of test triangles inside one scatterer, sized for a bounded buffer
  const double budget = SLAB_BUDGET;
  const double row_bytes = 3.0 * 2 * sizeof(M) * 2;  // per test triangle per union column, S and C
  std::vector<std::pair<int, int>> slabs;  // (t0, t1)
  for (auto& s : c->sc) {
    int per = int(std::max(1.0, budget / (row_bytes * (c->E_tot + s.topo.E))));
    per = std::min(per, s.topo.F);
    for (int t0 = 0; t0 < s.topo.F; t0 += per) slabs.push_back({s.tri_off + t0, s.tri_off + std::min(s.topo.F, t0 + per)});
  }
  const bool slabs_cached = (c->slabs == slabs && c->slab_elem == sizeof(M));
  if (!slabs_cached) {
    c->slabs = slabs;
    c->slab_elem = sizeof(M);
    c->slab_rows.clear();
    c->slab_rows_l.clear();
    c->slab_sp.clear();
    c->slab_sm.clear();
    c->slab_cs.clear();
    c->slab_nrows.clear();
  }
  int max_slab = 0, max_Em = 0;
  for (auto& sl : slabs) max_slab = std::max(max_slab, sl.second - sl.first);
  for (auto& s : c->sc) max_Em = std::max(max_Em, s.topo.E);
  DBuf HeS = dalloc_c<M>(c, size_t(2) * 3 * max_slab * c->E_tot),
       HeC = dalloc_c<M>(c, size_t(2) * 3 * max_slab * c->E_tot);
  DBuf HiS = dalloc_c<M>(c, size_t(2) * 3 * max_slab * max_Em), HiC = dalloc_c<M>(c, size_t(2) * 3 * max_slab * max_Em);
  HalfJob<M> hj{};
  hj.chunk_e = c->chunk_e.as<int32_t>();
  hj.chunk_ptr = c->chunk_ptr.as<int32_t>();
  hj.chunk_tri = c->chunk_tri.as<int32_t>();
  hj.edge_map = c->edge_map.as<int16_t>();
  hj.edge_scat = c->edge_scat_d.as<int32_t>();
  hj.E_tot = c->E_tot;
  hj.He_S = HeS.as<M>();
  hj.He_C = HeC.as<M>();
  hj.Hi_S = HiS.as<M>();
  hj.Hi_C = HiC.as<M>();
  hj.skip_lower = symform ? 1 : 0;
  hj.t1_tmin = c->t1_tmin.as<int32_t>();
  hj.ch_tmax = c->ch_tmax.as<int32_t>();
  // per union edge: T+ / T- (for the slot rows of pass 2)
  std::vector<int32_t> etp(c->E_tot), etm(c->E_tot), eap(c->E_tot), eam(c->E_tot);
  for (auto& s : c->sc)
    for (int f = 0; f < s.topo.F; ++f)
      for (int a = 0; a < 3; ++a) {
        const int e = s.edge_off + s.topo.t2e[3 * f + a];
        if (s.topo.sgn[3 * f + a] > 0) {
          etp[e] = s.tri_off + f;
          eap[e] = a;
        } else {
          etm[e] = s.tri_off + f;
          eam[e] = a;
        }
      }
  // one slab per scatterer: pass 2 writes every row of every block once, so
  // it overwrites (and zeroes the padding columns) instead of adding to
  // cleared matrices
  const bool overwrite = slabs.size() == c->sc.size();
  if (!overwrite) {
    zero(c->Se);
    zero(c->Ce);
    for (auto& b : c->Si) zero(b);
    for (auto& b : c->Ci) zero(b);
  }
  double ms_pass1 = 0.0, ms_pass2 = 0.0;
  EvTimer all(c->stream);
  for (auto& sl : slabs) {
    const int t0 = sl.first, t1 = sl.second;
    int m = 0;
    while (m + 1 < int(c->sc.size()) && c->sc[m + 1].tri_off <= t0) ++m;
    const Scat& s = c->sc[m];
    hj.slab_t0 = t0;
    hj.ld_i = s.topo.E;
    hj.edge_off_i = s.edge_off;
    {
      EvTimer t(c->stream);
      if (sizeof(M) == 8)
        launch_regular_rows<double, M>(p, hj, t0, t1, c->nchunks, c->max_list, c->stream);
      else
        launch_regular_rows<float, M>(p, hj, t0, t1, c->nchunks, c->max_list, c->stream);
      HIPCHK(hipGetLastError());
      ms_pass1 += t.stop();
    }
    // rows touched by this slab: edges of scatterer m with T+ or T- inside
    const size_t si = size_t(&sl - &slabs[0]);
    if (!slabs_cached) {
      std::vector<int32_t> rows, sp, smn, rows_l, cs;
      for (int e = s.edge_off; e < s.edge_off + s.topo.E; ++e) {
        const bool ip = etp[e] >= t0 && etp[e] < t1, im = etm[e] >= t0 && etm[e] < t1;
        if (!ip && !im) continue;
        rows.push_back(e);
        rows_l.push_back(e - s.edge_off);
        sp.push_back(ip ? 3 * (etp[e] - t0) + eap[e] : -1);
        smn.push_back(im ? 3 * (etm[e] - t0) + eam[e] : -1);
        cs.push_back((e - s.edge_off) / SYM_T * SYM_T);  // first column of the row's upper tiles
      }
      c->slab_rows.push_back(upload(c, rows));
      c->slab_rows_l.push_back(upload(c, rows_l));
      c->slab_sp.push_back(upload(c, sp));
      c->slab_sm.push_back(upload(c, smn));
      c->slab_cs.push_back(upload(c, cs));
      c->slab_nrows.push_back(int(rows.size()));
    }
    DBuf &drows = c->slab_rows[si], &drl = c->slab_rows_l[si], &dsp = c->slab_sp[si], &dsm = c->slab_sm[si];
    const int32_t* dcs = symform ? c->slab_cs[si].as<int32_t>() : nullptr;
    const int nr = c->slab_nrows[si];
    {
      EvTimer t(c->stream);
      launch_rows_combine<M>(c->Se.as<M>(), c->ldE, HeS.as<M>(), c->E_tot, drows.as<int32_t>(), dsp.as<int32_t>(),
                             dsm.as<int32_t>(), nr, c->E_tot, c->stream, overwrite, dcs);
      launch_rows_combine<M>(c->Ce.as<M>(), c->ldE, HeC.as<M>(), c->E_tot, drows.as<int32_t>(), dsp.as<int32_t>(),
                             dsm.as<int32_t>(), nr, c->E_tot, c->stream, overwrite, dcs);
      launch_rows_combine<M>(c->Si[m].as<M>(), c->ldI[m], HiS.as<M>(), s.topo.E, drl.as<int32_t>(), dsp.as<int32_t>(),
                             dsm.as<int32_t>(), nr, s.topo.E, c->stream, overwrite, dcs);
      launch_rows_combine<M>(c->Ci[m].as<M>(), c->ldI[m], HiC.as<M>(), s.topo.E, drl.as<int32_t>(), dsp.as<int32_t>(),
                             dsm.as<int32_t>(), nr, s.topo.E, c->stream, overwrite, dcs);
      HIPCHK(hipGetLastError());
      ms_pass2 += t.stop();
    }
  }
  c->prof.ms_assemble_regular = ms_pass1;
  c->prof.ms_regular_combine = ms_pass2;
  c->prof.regular_launches = int(slabs.size());
  // the FP64 singular blocks, kept for the matrix-free FP64 product
  realloc_c<double>(c, c->sing.blk, size_t(std::max<int64_t>(c->sing.npairs, 1)) * 72);
  sp_.blk = c->sing.blk.as<double>();
  sp_.e_row = c->sing.e_row.as<int32_t>();
  sp_.e_col = c->sing.e_col.as<int32_t>();
  sp_.e_iptr = c->sing.e_iptr.as<int64_t>();
  sp_.e_item = c->sing.e_item.as<int32_t>();
  sp_.e_nnz = c->sing.e_nnz;
  {
    EvTimer t(c->stream);
    launch_singular<M>(p, sp_, c->stream);
    HIPCHK(hipGetLastError());
    c->prof.ms_assemble_singular = t.stop();
  }
  c->comb = false;
  c->sym.ready = false;
  c->AC = DBuf();
  c->AS1 = DBuf();
  c->AS2 = DBuf();
  for (bool& st : c->sym.lower_stale) st = symform;
  if (c->sc.size() == 1 && c->comb_ok) {  // three combined matrices for the operator products
    if (symform) {
      const Scat& s = c->sc[0];
      {
        const double wt = wall_ms();
        const bool fresh = c->sym.n != int(E);
        sym_tables(c);
        if (fresh) c->prof.wall_tables_A += wall_ms() - wt;
      }
      realloc_c<M>(c, c->sym.pack, size_t(c->sym.ntiles) * 3 * SYM_T * SYM_T * 2);
      realloc_c<M>(c, c->sym.val, size_t(std::max<int64_t>(c->sym.nnz, 1)) * 6);
      realloc_c<double>(c, c->sym.part, size_t(c->sym.nt) * c->sym.nt * SYM_T * 4);
      launch_pack_sym3<M>(c->Se.as<M>(), c->Ce.as<M>(), c->Si[0].as<M>(), c->Ci[0].as<M>(), c->ldE, int(E),
                          c->sym.tij.as<int32_t>(), c->sym.ntiles, c->k_ext, s.k.real(), s.k.imag(),
                          c->sym.pack.as<M>(), c->stream);
      launch_sym_corr_sing<M>(c->sym.iptr.as<int64_t>(), c->sym.item.as<int32_t>(), c->sing.blk.as<double>(),
                              c->sym.nnz, c->k_ext, s.k.real(), s.k.imag(), c->sym.val.as<M>(), c->stream);
      HIPCHK(hipGetLastError());
      c->sym.ready = true;
    } else {
      build_comb<M>(c);
    }
  } else {
    c->sym.pack = DBuf();
    c->sym.val = DBuf();
    c->sym.part = DBuf();
  }
  c->prof.ms_assemble_A = all.stop();
  c->prof.recompute = c->recompute;
  // work counters: disjoint ordered pairs by class (same rule as the
  // kernel); pure metadata of the mesh and the rule orders, kept across
  // assemblies of the same geometry
  const int64_t ckey = (int64_t(c->F_tot) << 12) | (o.q_near << 8) | (o.q_medium << 4) | o.q_far;
  int64_t reg_pairs = 0, reg_pts = 0;
  if (c->count_key == ckey) {
    reg_pairs = c->count_pairs;
    reg_pts = c->count_pts;
  } else {
    const double wt = wall_ms();
    // exact count over all unordered pairs on the device, with the class rule
    // of the regular kernel
    const int np[5] = {0, 1, 3, 4, 6};
    DBuf cntd = dalloc_c<int64_t>(c, 2);
    launch_cls_set_i64(cntd.as<int64_t>(), 0, c->stream);
    launch_cls_set_i64(cntd.as<int64_t>() + 1, 0, c->stream);
    launch_count_regular(c->F_tot, c->tcen.as<double>(), c->tdiam2.as<double>(), c->tvid.as<int32_t>(), np[o.q_near],
                         np[o.q_medium], np[o.q_far], reinterpret_cast<unsigned long long*>(cntd.p), c->stream);
    HIPCHK(hipGetLastError());
    read_scalars(c, {{&reg_pairs, {cntd.as<int64_t>(), 8}}, {&reg_pts, {cntd.as<int64_t>() + 1, 8}}});
    c->prof.wall_tables_A += wall_ms() - wt;
    c->count_key = ckey;
    c->count_pairs = reg_pairs;
    c->count_pts = reg_pts;
  }
  c->prof.regular_pairs = reg_pairs;
  c->prof.regular_point_pairs = reg_pts;
  c->prof.singular_pairs = sp_.npairs;
  c->prof.singular_point_pairs = npts_sing;
  c->prof.n_wavenumbers = 2;
}

// ---------------------------------------------------------------------------
// Dual cells and near-field BC operators of P
// ---------------------------------------------------------------------------

void build_duals(pmchwt_ctx* c) {
  int cell_off = 0, child_off = 0, bvert_off = 0;
  for (auto& s : c->sc) {
    if (!s.dual_built) {
      std::string err;
      if (!build_dual(s.topo, s.dual, err)) throw Fail{PMCHWT_ERR_INVALID_MESH, err};
      if (s.dual.max_valence > 16) throw Fail{PMCHWT_ERR_INVALID_MESH, "vertex valence above 16"};
      s.dual_built = true;
    }
    s.cell_off = cell_off;
    s.child_off = child_off;
    s.bvert_off = bvert_off;
    cell_off += s.topo.nv;
    child_off += 6 * s.topo.F;
    bvert_off += s.dual.nbv;
  }
}

void upload_cells(pmchwt_ctx* c, CellDev& d) {
  // sizes first, then every table filled by index (bulk copies with offsets)
  size_t ncell = 0, nchild = 0, nring = 0, ninc = 0, nrec = 0, E = 0;
  for (const Scat& s : c->sc) {
    ncell += size_t(s.topo.nv);
    nchild += 6 * size_t(s.topo.F);
    nring += size_t(s.dual.cell_ptr[s.topo.nv]);
    ninc += size_t(s.dual.inc_ptr[s.topo.nv]);
    nrec += size_t(s.dual.coef_ptr[s.topo.nv]);
    E += size_t(s.topo.E);
  }
  std::vector<int32_t> cell_ptr(ncell + 1), ring(nring), child_vid(3 * nchild), cell_scat(ncell), child_cell(nchild),
      child_pos(nchild), child_parent(nchild), inc_ptr(ncell + 1), inc_edges(ninc), edge_scat(E), eoff;
  std::vector<double> child_v(9 * nchild), child_cen(3 * nchild), child_diam2(nchild), child_area(nchild),
      coef(4 * nrec);
  std::vector<int64_t> coef_ptr(ncell + 1);
  cell_ptr[0] = 0;
  inc_ptr[0] = 0;
  coef_ptr[0] = 0;
  size_t ring0 = 0, inc0 = 0, rec0 = 0;
  for (size_t m = 0; m < c->sc.size(); ++m) {
    const Scat& s = c->sc[m];
    const DualCells& D = s.dual;
    const Topo& T = s.topo;
    eoff.push_back(s.edge_off);
    std::fill(edge_scat.begin() + s.edge_off, edge_scat.begin() + s.edge_off + T.E, int32_t(m));
    for (int ch = 0; ch < 6 * T.F; ++ch) {
      const size_t g = size_t(s.child_off + ch);
      double P[3][3];
      for (int k = 0; k < 3; ++k) {
        const int id = D.child_vid[3 * size_t(ch) + k];
        child_vid[3 * g + k] = s.bvert_off + id;
        for (int dd = 0; dd < 3; ++dd) {
          P[k][dd] = D.bv[3 * size_t(id) + dd];
          child_v[9 * g + 3 * k + dd] = P[k][dd];
        }
      }
      for (int dd = 0; dd < 3; ++dd) child_cen[3 * g + dd] = (P[0][dd] + P[1][dd] + P[2][dd]) / 3.0;
      double mm = 0;
      const int pr[3][2] = {{0, 1}, {1, 2}, {2, 0}};
      for (auto& q : pr) {
        const double ex = P[q[0]][0] - P[q[1]][0], ey = P[q[0]][1] - P[q[1]][1], ez = P[q[0]][2] - P[q[1]][2];
        mm = std::max(mm, ex * ex + ey * ey + ez * ez);
      }
      child_diam2[g] = mm;
      const double u[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
      const double w[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
      const double cr[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
      child_area[g] = 0.5 * std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
      child_parent[g] = s.tri_off + ch / 6;
    }
    for (int v = 0; v < T.nv; ++v) {
      const size_t cv = size_t(s.cell_off + v);
      const int r0 = D.cell_ptr[v], n2 = D.cell_ptr[v + 1] - r0;
      for (int i = 0; i < n2; ++i) {
        const int ch = D.ring[size_t(r0) + i];
        ring[ring0 + size_t(r0) + i] = s.child_off + ch;
        child_cell[size_t(s.child_off + ch)] = int32_t(cv);
        child_pos[size_t(s.child_off + ch)] = i;
      }
      cell_ptr[cv + 1] = int32_t(ring0) + D.cell_ptr[v + 1];
      inc_ptr[cv + 1] = int32_t(inc0) + D.inc_ptr[v + 1];
      coef_ptr[cv + 1] = int64_t(rec0) + D.coef_ptr[v + 1];
      cell_scat[cv] = int32_t(m);
    }
    for (int q = 0; q < D.inc_ptr[T.nv]; ++q) inc_edges[inc0 + size_t(q)] = s.edge_off + D.inc_edges[q];
    std::copy(D.coef.begin(), D.coef.begin() + 4 * D.coef_ptr[T.nv], coef.begin() + 4 * rec0);
    ring0 += size_t(D.cell_ptr[T.nv]);
    inc0 += size_t(D.inc_ptr[T.nv]);
    rec0 += size_t(D.coef_ptr[T.nv]);
  }
  d.ncell = int(ncell);
  d.nchild = int(nchild);
  d.cell_ptr = upload(c, cell_ptr);
  d.ring = upload(c, ring);
  d.child_v = upload(c, child_v);
  d.child_vid = upload(c, child_vid);
  d.child_cen = upload(c, child_cen);
  d.child_diam2 = upload(c, child_diam2);
  d.child_area = upload(c, child_area);
  d.coef_ptr = upload(c, coef_ptr);
  d.coef = upload(c, coef);
  d.cell_scat = upload(c, cell_scat);
  d.child_cell = upload(c, child_cell);
  d.child_pos = upload(c, child_pos);
  d.child_parent = upload(c, child_parent);
  d.inc_ptr = upload(c, inc_ptr);
  d.inc_edges = upload(c, inc_edges);
  d.edge_scat = upload(c, edge_scat);
  d.edge_off = upload(c, eoff);
}

void build_nearfield_tables(pmchwt_ctx* c, double chi, bool cross, const CellDev& cells);
void run_nearfield_kernel(pmchwt_ctx* c, const pmchwt_assembly_opts& o, CellDev& cells);

void assemble_P_impl(pmchwt_ctx* c, const pmchwt_assembly_opts& o, int kind, CellDev& cells) {
  c->PSi.release();
  c->PCi.release();
  c->PSe.release();
  c->PCe.release();
  c->PSi32.release();
  c->PCi32.release();
  c->PSe32.release();
  c->PCe32.release();
  c->bsrPi.clear();
  c->bsrPe = BsrHold();
  c->precond = kind;
  c->P_int = (kind == PMCHWT_P_A || kind == PMCHWT_P_D || kind == PMCHWT_P_D_INT || kind == PMCHWT_P_S_INT);
  c->P_ext = (kind == PMCHWT_P_A || kind == PMCHWT_P_D || kind == PMCHWT_P_D_EXT || kind == PMCHWT_P_S_EXT);
  c->P_C = !(kind == PMCHWT_P_S_INT || kind == PMCHWT_P_S_EXT);
  c->P_cross = (kind == PMCHWT_P_A && c->sc.size() > 1);
  c->nnzP = 0;
  c->prof.ms_assemble_P = 0;
  c->prof.bary_pairs = 0;
  if (kind == PMCHWT_P_I) return;
  const double chi = o.chi < 0 ? -1.0 : o.chi;
  if (!(c->nf.valid && c->nf.chi == chi && c->nf.cross == c->P_cross)) {
    const double wt = wall_ms();
    build_nearfield_tables(c, chi, c->P_cross, cells);
    c->prof.wall_tables_P += wall_ms() - wt;
    c->nf.valid = true;
    c->nf.chi = chi;
    c->nf.cross = c->P_cross;
  }
  c->nnzP = c->nf.nnz;
  c->prof.bary_pairs = c->nf.bary_pairs;
  auto vals = [&](DBuf& b) {  // every entry is written by the gather of the near-field kernel
    realloc_c<double>(c, b, 2 * size_t(std::max<int64_t>(c->nnzP, 1)));
  };
  if (c->P_int) {
    vals(c->PSi);
    if (c->P_C) vals(c->PCi);
  }
  if (c->P_ext) {
    vals(c->PSe);
    if (c->P_C) vals(c->PCe);
  }
  run_nearfield_kernel(c, o, cells);
  if (o.precision == PMCHWT_MIXED) {
    auto f32 = [&](const DBuf& src, DBuf& dst) {
      if (!src.p) return;
      dst = dalloc_c<float>(c, 2 * size_t(std::max<int64_t>(c->nnzP, 1)));
      launch_d2f(src.as<double>(), dst.as<float>(), 2 * c->nnzP, c->stream);
    };
    f32(c->PSi, c->PSi32);
    f32(c->PCi, c->PCi32);
    f32(c->PSe, c->PSe32);
    f32(c->PCe, c->PCe32);
    HIPCHK(hipGetLastError());
  }
}

// Near-field pattern of P (entries (i, j), i and j in one scatterer unless
// `cross`, whose BC support boxes are within chi; chi < 0 keeps all) and the
// dual-cell pair tables of its kernel, built by the classification kernels.
// The host only lays out the per-edge boxes and end cells (O(E)) and sizes
// the grid and the outputs.
void build_nearfield_tables(pmchwt_ctx* c, double chi, bool cross, const CellDev& cells) {
  const int E = c->E_tot;
  hipStream_t st = c->stream;
  std::vector<double> box(6 * size_t(E));
  std::vector<int32_t> escat(E), ecell(2 * size_t(E)), sc_first, sc_n;
  double ext = 0.0, gmin[3] = {1e300, 1e300, 1e300}, gmax[3] = {-1e300, -1e300, -1e300};
  for (size_t m = 0; m < c->sc.size(); ++m) {
    const Scat& s = c->sc[m];
    for (int e = 0; e < s.topo.E; ++e) {
      const size_t g = size_t(s.edge_off + e);
      for (int q = 0; q < 6; ++q) box[6 * g + q] = s.dual.bbox[6 * size_t(e) + q];
      for (int d = 0; d < 3; ++d) {
        const double lo = box[6 * g + d], hi = box[6 * g + 3 + d], ce = 0.5 * (lo + hi);
        ext = std::max(ext, hi - lo);
        gmin[d] = std::min(gmin[d], ce);
        gmax[d] = std::max(gmax[d], ce);
      }
      escat[g] = int32_t(m);
      ecell[2 * g] = s.cell_off + s.topo.edges[2 * size_t(e)];
      ecell[2 * g + 1] = s.cell_off + s.topo.edges[2 * size_t(e) + 1];
    }
    sc_first.push_back(s.edge_off);
    sc_n.push_back(s.topo.E);
  }
  DBuf d_box = upload(c, box), d_escat = upload(c, escat), d_ecell = upload(c, ecell);
  DBuf cnt = dalloc_c<int32_t>(c, size_t(E)), stats = dalloc_c<int32_t>(c, 4);
  DBuf rowptr = dalloc_c<int64_t>(c, size_t(E) + 1);
  launch_cls_fill_i32(stats.as<int32_t>(), 4, 0, st);
  DBuf d_first = upload(c, sc_first), d_n = upload(c, sc_n);
  DBuf gcell, gcnt, gstart, gitem;
  NfJob J{};
  if (chi < 0) {
    launch_nf_dense(E, d_escat.as<int32_t>(), d_first.as<int32_t>(), d_n.as<int32_t>(), cross ? 1 : 0,
                    cnt.as<int32_t>(), stats.as<int32_t>(), st);
  } else {
    // cells of at least chi + the largest box extent (slightly enlarged against
    // rounding), coarsened until there are at most about 2 E of them
    NfGrid g{};
    double h = (chi + ext) * (1.0 + 1e-9) + 1e-300;
    int64_t ncells = 0;
    for (;;) {
      ncells = 1;
      for (int d = 0; d < 3; ++d) {
        g.dims[d] = int(std::max(1.0, std::min(1024.0, std::floor((gmax[d] - gmin[d]) / h) + 1.0)));
        ncells *= g.dims[d];
      }
      if (ncells <= 2 * int64_t(E) + 64) break;
      h *= 1.25;
    }
    for (int d = 0; d < 3; ++d) g.gmin[d] = gmin[d];
    g.h = h;
    gcell = dalloc_c<int32_t>(c, size_t(E));
    gcnt = dalloc_c<int32_t>(c, size_t(ncells));
    gstart = dalloc_c<int64_t>(c, size_t(ncells) + 1);
    gitem = dalloc_c<int32_t>(c, size_t(E));
    launch_cls_fill_i32(gcnt.as<int32_t>(), ncells, 0, st);
    launch_nf_bin(d_box.as<double>(), E, g, gcell.as<int32_t>(), gcnt.as<int32_t>(), st);
    launch_scan_i32(gcnt.as<int32_t>(), int(ncells), gstart.as<int64_t>(), st);
    launch_cls_fill_i32(gcnt.as<int32_t>(), ncells, 0, st);
    launch_nf_bin_fill(gcell.as<int32_t>(), E, gstart.as<int64_t>(), gcnt.as<int32_t>(), gitem.as<int32_t>(), st);
    J.E = E;
    J.box = d_box.as<double>();
    J.escat = d_escat.as<int32_t>();
    J.g = g;
    J.gcell = gcell.as<int32_t>();
    J.gstart = gstart.as<int64_t>();
    J.gitem = gitem.as<int32_t>();
    J.chi = chi;
    J.cross = cross ? 1 : 0;
    launch_nf_count(J, cnt.as<int32_t>(), stats.as<int32_t>(), st);
  }
  launch_scan_i32(cnt.as<int32_t>(), E, rowptr.as<int64_t>(), st);
  HIPCHK(hipGetLastError());
  int64_t nnz = 0;
  int32_t maxc = 0;
  read_scalars(c, {{&nnz, {rowptr.as<int64_t>() + E, 8}}, {&maxc, {stats.as<int32_t>(), 4}}});
  if (chi >= 0 && maxc > nf_row_capacity())
    throw Fail{PMCHWT_ERR_INVALID_ARG, "near-field cutoff keeps " + std::to_string(maxc) +
                                           " entries in one row of P (at most " + std::to_string(nf_row_capacity()) +
                                           "): chi too large for a sparse preconditioner"};
  DBuf col = dalloc_c<int32_t>(c, size_t(std::max<int64_t>(nnz, 1)));
  if (chi < 0)
    launch_nf_dense_fill(E, d_escat.as<int32_t>(), d_first.as<int32_t>(), cross ? 1 : 0, rowptr.as<int64_t>(),
                         col.as<int32_t>(), st);
  else
    launch_nf_fill(J, rowptr.as<int64_t>(), pow2_ceil(std::max(maxc, 1)), col.as<int32_t>(), st);
  HIPCHK(hipGetLastError());
  c->p_rowptr = std::move(rowptr);
  c->p_col = std::move(col);
  c->nf.nnz = nnz;
  c->nf.host_valid = false;
  c->h_rowptr.clear();
  c->h_col.clear();
  // dual-cell pairs: count, scan, fill
  const int ncell = cells.ncell;
  DBuf ncw = dalloc_c<int32_t>(c, size_t(ncell)), nslot = dalloc_c<int32_t>(c, size_t(ncell));
  DBuf pairoff = dalloc_c<int64_t>(c, size_t(ncell) + 1), slotbase = dalloc_c<int64_t>(c, size_t(ncell) + 1);
  CellPairJob P{};
  P.inc_ptr = cells.inc_ptr.as<int32_t>();
  P.inc_edges = cells.inc_edges.as<int32_t>();
  P.rowptr = c->p_rowptr.as<int64_t>();
  P.col = c->p_col.as<int32_t>();
  P.ecell = d_ecell.as<int32_t>();
  P.ncw = ncw.as<int32_t>();
  P.nslot = nslot.as<int32_t>();
  P.flag = stats.as<int32_t>() + 1;
  launch_cell_pairs(P, ncell, false, st);
  launch_scan_i32(ncw.as<int32_t>(), ncell, pairoff.as<int64_t>(), st);
  launch_scan_i32(nslot.as<int32_t>(), ncell, slotbase.as<int64_t>(), st);
  HIPCHK(hipGetLastError());
  int64_t npairs = 0, nslots = 0;
  int32_t over = 0;
  read_scalars(c, {{&npairs, {pairoff.as<int64_t>() + ncell, 8}},
                   {&nslots, {slotbase.as<int64_t>() + ncell, 8}},
                   {&over, {stats.as<int32_t>() + 1, 4}}});
  if (over)
    throw Fail{PMCHWT_ERR_INVALID_ARG, "near-field cutoff joins a dual cell to more than " +
                                           std::to_string(cell_pair_capacity()) +
                                           " others: chi too large for a sparse preconditioner"};
  c->nf.cpairs = dalloc_c<int32_t>(c, size_t(2 * std::max<int64_t>(npairs, 1)));
  c->nf.slot_off = dalloc_c<int64_t>(c, size_t(npairs) + 1);
  c->nf.slot_pos = dalloc_c<int64_t>(c, size_t(std::max<int64_t>(nslots, 1)));
  c->nf.entry_slots = dalloc_c<int64_t>(c, 4 * size_t(std::max<int64_t>(nnz, 1)));
  launch_cls_fill_i32(reinterpret_cast<int32_t*>(c->nf.entry_slots.p), 8 * std::max<int64_t>(nnz, 1), -1, st);
  P.entry_slots = c->nf.entry_slots.as<int64_t>();
  P.pairoff = pairoff.as<int64_t>();
  P.slotbase = slotbase.as<int64_t>();
  P.cpairs = c->nf.cpairs.as<int32_t>();
  P.slot_off = c->nf.slot_off.as<int64_t>();
  P.slot_pos = c->nf.slot_pos.as<int64_t>();
  launch_cell_pairs(P, ncell, true, st);
  launch_cls_set_i64(c->nf.slot_off.as<int64_t>() + npairs, nslots, st);
  HIPCHK(hipGetLastError());
  c->nf.bary_pairs = 4 * nslots;  // 4 barycentric pairs per (slot of v) x (slot of w)
  c->nf.nslots = nslots;
  c->nf.npairs = npairs;
  HIPCHK(hipStreamSynchronize(st));  // the host inputs above go out of scope
}

// Host copy of the pattern of P, for the block and entry accessors.
void host_pattern(pmchwt_ctx* c) {
  if (c->nf.host_valid) return;
  c->h_rowptr.resize(size_t(c->E_tot) + 1);
  c->h_col.resize(size_t(c->nf.nnz));
  HIPCHK(hipMemcpyAsync(c->h_rowptr.data(), c->p_rowptr.p, c->h_rowptr.size() * 8, hipMemcpyDeviceToHost, c->stream));
  if (c->nf.nnz > 0)
    HIPCHK(hipMemcpyAsync(c->h_col.data(), c->p_col.p, c->h_col.size() * 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->nf.host_valid = true;
}

void run_nearfield_kernel(pmchwt_ctx* c, const pmchwt_assembly_opts& o, CellDev& cells) {
  SSTables ss;
  build_ss(c, o.n_singular, ss);
  BCJob j{};
  j.npairs = c->nf.npairs;
  j.cpairs = c->nf.cpairs.as<int32_t>();
  j.slot_off = c->nf.slot_off.as<int64_t>();
  j.slot_pos = c->nf.slot_pos.as<int64_t>();
  j.want_int = c->P_int;
  j.want_ext = c->P_ext;
  j.want_C = c->P_C;
  j.fp32 = o.precision == PMCHWT_MIXED;  // mixed-precision P: FP32 integrals, FP64 entries
  j.k_int = c->k_int.as<double>();
  j.k_ext = c->k_ext;
  j.q_near = o.q_near;
  j.q_medium = o.q_medium;
  j.q_far = o.q_far;
  j.n_sing = o.n_singular;
  for (int k = 1; k <= 3; ++k) {
    j.tab[k] = ss.tab[k].as<double>();
    j.npts[k] = ss.npts[k];
  }
  j.out_Si = c->PSi.as<double>();
  j.out_Ci = c->PCi.as<double>();
  j.out_Se = c->PSe.as<double>();
  j.out_Ce = c->PCe.as<double>();
  j.nv = 2 * ((c->P_int ? 1 : 0) + (c->P_ext ? 1 : 0)) * (c->P_C ? 2 : 1);
  DBuf sv = dalloc_c<double>(c, size_t(std::max<int64_t>(c->nf.nslots, 1)) * size_t(j.nv));
  j.slot_val = sv.as<double>();
  j.entry_slots = c->nf.entry_slots.as<int64_t>();
  j.nnz = c->nf.nnz;
  j.nslots = c->nf.nslots;
  EvTimer t(c->stream);
  if (j.npairs > 0) {
    launch_bc_nearfield(asm_params<double>(c), cells.params(), j, c->stream);
    launch_bc_gather(j, c->stream);
  }
  HIPCHK(hipGetLastError());
  c->prof.ms_assemble_P = t.stop();
  c->prof.nnz_P = c->nnzP;
}

void rocsolver_check(rocblas_status s, const char* what) {
  if (s != rocblas_status_success) throw Fail{PMCHWT_ERR_DEVICE, std::string(what) + " failed"};
}

// In-place inverse of a column-major n x n matrix by blocked Gauss-Jordan
// elimination without pivoting: per 128-wide pivot block, the block inverse
// (one-workgroup kernel) and two rocBLAS GEMMs (row-block scaling and the
// rank-128 update of the whole matrix).  Stable here because the symmetric
// part of the mixed mass matrix is positive definite.
// In-place blocked Gauss-Jordan inverse of the column-major n x n matrix X
// (no pivoting: the mixed mass matrix has a positive definite symmetric
// part).  With look-ahead: as soon as the next pivot column block has been
// updated, its small block inverse runs on the side stream while the main
// stream performs the rank update of the other columns.
void gj_inverse(pmchwt_ctx* c, double* X, int n) {
  const int B = 128;
  DBuf Pinv[2] = {dalloc_c<double>(c, size_t(B) * B), dalloc_c<double>(c, size_t(B) * B)};
  DBuf Cc[2] = {dalloc_c<double>(c, size_t(n) * B), dalloc_c<double>(c, size_t(n) * B)};
  DBuf R = dalloc_c<double>(c, size_t(B) * n);
  const double one = 1.0, zero = 0.0, mone = -1.0;
  auto prepare = [&](int p0, int slot, hipStream_t st) {
    const int b = std::min(B, n - p0);
    launch_gj_block_inverse(X + int64_t(p0) * n + p0, n, Pinv[slot].as<double>(), b, st);
    launch_gj_take_columns(X, n, p0, b, Cc[slot].as<double>(), st);
  };
  auto update = [&](int slot, int b, int j0, int nj) {  // X[:, j0:j0+nj] -= C R[:, j0:j0+nj]
    if (nj <= 0) return;
    rocsolver_check(rocblas_dgemm(c->blas, rocblas_operation_none, rocblas_operation_none, n, nj, b, &mone,
                                  Cc[slot].as<double>(), n, R.as<double>() + int64_t(j0) * b, b, &one,
                                  X + int64_t(j0) * n, n),
                    "rocblas_dgemm(rank update)");
  };
  auto put_rows = [&](int p0, int b, int j0, int nj) {  // X[p0:p0+b, j0:j0+nj] = R[:, j0:j0+nj]
    if (nj <= 0) return;
    HIPCHK(hipMemcpy2DAsync(X + int64_t(j0) * n + p0, size_t(n) * 8, R.as<double>() + int64_t(j0) * b,
                            size_t(b) * 8, size_t(b) * 8, size_t(nj), hipMemcpyDeviceToDevice, c->stream));
  };
  prepare(0, 0, c->stream);
  int slot = 0;
  for (int p0 = 0; p0 < n; p0 += B) {
    const int b = std::min(B, n - p0);
    const int q0 = p0 + b, bq = std::min(B, n - q0);
    rocsolver_check(rocblas_dgemm(c->blas, rocblas_operation_none, rocblas_operation_none, b, n, b, &one,
                                  Pinv[slot].as<double>(), b, X + p0, n, &zero, R.as<double>(), b),
                    "rocblas_dgemm(row block)");
    if (bq > 0) {
      update(slot, b, q0, bq);
      put_rows(p0, b, q0, bq);
      HIPCHK(hipEventRecord(c->ev_main, c->stream));
      HIPCHK(hipStreamWaitEvent(c->side, c->ev_main, 0));
      prepare(q0, slot ^ 1, c->side);
      HIPCHK(hipEventRecord(c->ev_side, c->side));
    }
    const int nl = bq > 0 ? q0 : n;
    update(slot, b, 0, nl);
    update(slot, b, q0 + bq, n - q0 - bq);
    put_rows(p0, b, 0, nl);
    put_rows(p0, b, q0 + bq, n - q0 - bq);
    if (bq > 0) HIPCHK(hipStreamWaitEvent(c->stream, c->ev_side, 0));
    slot ^= 1;
  }
  // look-ahead steps are joined into the stream; temporaries return to the pool
}

// y (rows x Nr, row-major, ldy) = [y -] A (rows x K, row-major, lda) B^T
// (B: Nr x K row-major) with rocBLAS SGEMM on the context's stream: a plain
// GEMM, where the library's FP32 matrix-core kernels outrun the fused product
// kernel at K = 128 (about 100 vs 73 TFLOP/s on the 7680 x 7680 update).
void sgemm_abt(pmchwt_ctx* c, const float* A, int64_t lda, const float* Bm, int K, int rows, int Nr, float* y,
               int64_t ldy, bool subtract) {
  const float alpha = subtract ? -1.0f : 1.0f, beta = subtract ? 1.0f : 0.0f;
  // column-major view: y^T (Nr x rows) = B (Nr x K) A^T, i.e. op(B-as-stored) = T
  rocsolver_check(rocblas_sgemm(c->blas, rocblas_operation_transpose, rocblas_operation_none, Nr, rows, K, &alpha, Bm,
                                K, A, int(lda), &beta, y, int(ldy)),
                  "rocblas_sgemm");
}

// The same inverse in FP32 on the matrix cores (rank updates by SGEMM) (n a multiple of 32, so that
// every pivot block is a multiple of the 32-wide K tile).  Pivot blocks are
// inverted row-major and the taken columns stored row-major, so that both
// products are A B^T with K contiguous:
//   R (n x b, = the b x n row block Pinv X[p,:] read column-major) = X[p,:]^T Pinv^T,
//   X[:, J] -= C R[:, J]  as  (X^T)[J, :] -= R[J, :] C^T.
void gj_inverse_f32(pmchwt_ctx* c, float* X, int n) {
  const int B = 128;
  DBuf Pinv[2] = {dalloc_c<float>(c, size_t(B) * B), dalloc_c<float>(c, size_t(B) * B)};
  DBuf Cc[2] = {dalloc_c<float>(c, size_t(n) * B), dalloc_c<float>(c, size_t(n) * B)};
  DBuf R = dalloc_c<float>(c, size_t(B) * n);
  auto prepare = [&](int p0, int slot, hipStream_t st) {
    const int b = std::min(B, n - p0);
    launch_gj_block_inverse_f32(X + int64_t(p0) * n + p0, n, Pinv[slot].as<float>(), b, st);
    launch_gj_take_columns_f32(X, n, p0, b, Cc[slot].as<float>(), st);
  };
  auto update = [&](int slot, int b, int j0, int nj) {
    if (nj <= 0) return;
    sgemm_abt(c, R.as<float>() + int64_t(j0) * b, b, Cc[slot].as<float>(), b, nj, n, X + int64_t(j0) * n, n, true);
  };
  auto put_rows = [&](int p0, int b, int j0, int nj) {
    if (nj <= 0) return;
    HIPCHK(hipMemcpy2DAsync(X + int64_t(j0) * n + p0, size_t(n) * 4, R.as<float>() + int64_t(j0) * b, size_t(b) * 4,
                            size_t(b) * 4, size_t(nj), hipMemcpyDeviceToDevice, c->stream));
  };
  prepare(0, 0, c->stream);
  int slot = 0;
  for (int p0 = 0; p0 < n; p0 += B) {
    const int b = std::min(B, n - p0);
    const int q0 = p0 + b, bq = std::min(B, n - q0);
    sgemm_abt(c, X + p0, n, Pinv[slot].as<float>(), b, n, b, R.as<float>(), b, false);
    if (bq > 0) {
      update(slot, b, q0, bq);
      put_rows(p0, b, q0, bq);
      HIPCHK(hipEventRecord(c->ev_main, c->stream));
      HIPCHK(hipStreamWaitEvent(c->side, c->ev_main, 0));
      prepare(q0, slot ^ 1, c->side);
      HIPCHK(hipEventRecord(c->ev_side, c->side));
    }
    const int nl = bq > 0 ? q0 : n;
    update(slot, b, 0, nl);
    update(slot, b, q0 + bq, n - q0 - bq);
    put_rows(p0, b, 0, nl);
    put_rows(p0, b, q0 + bq, n - q0 - bq);
    if (bq > 0) HIPCHK(hipStreamWaitEvent(c->stream, c->ev_side, 0));
    slot ^= 1;
  }
  // every look-ahead step has been joined into the stream: the temporaries go
  // back to the pool without a host wait
  HIPCHK(hipGetLastError());
}

// RWG Gram pattern: row i holds edge i and the other edges of its two
// triangles (sorted, scatterer-local columns); g_pos maps local pair (a, b)
// of every triangle to its CSR slot.
void build_gram_pattern(pmchwt_ctx* c) {
  std::vector<int64_t> rowptr(size_t(c->E_tot) + 1, 0), pos(9 * size_t(c->F_tot));
  std::vector<int32_t> col;
  for (const Scat& s : c->sc) {
    const Topo& T = s.topo;
    for (int e = 0; e < T.E; ++e) {
      std::vector<int32_t> nb;
      for (int tt : {T.tplus[e], T.tminus[e]})
        for (int a = 0; a < 3; ++a) nb.push_back(T.t2e[3 * size_t(tt) + a]);
      std::sort(nb.begin(), nb.end());
      nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
      col.insert(col.end(), nb.begin(), nb.end());
      rowptr[size_t(s.edge_off) + e + 1] = int64_t(col.size());
    }
  }
  for (const Scat& s : c->sc) {
    const Topo& T = s.topo;
    for (int f = 0; f < T.F; ++f)
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          const int i = s.edge_off + T.t2e[3 * size_t(f) + a], jl = T.t2e[3 * size_t(f) + b];
          auto beg = col.begin() + rowptr[i], end = col.begin() + rowptr[i + 1];
          auto it = std::lower_bound(beg, end, jl);
          if (it == end || *it != jl) throw Fail{PMCHWT_ERR_INVALID_MESH, "Gram pattern inconsistent with topology"};
          pos[9 * size_t(s.tri_off + f) + 3 * a + b] = int64_t(it - col.begin());
        }
  }
  c->g_rowptr = upload(c, rowptr);
  c->g_col = upload(c, col);
  c->g_pos = upload(c, pos);
  c->g_val = dalloc<double>(col.size());
  c->gram_valid = true;
}

// M_A^-1 (row-major, n rows, leading dimension ld; padding columns zero,
// padding rows [n, ld) of an ld x ld X set to the identity) by the Chebyshev
// iteration of k_cheb_step (M's columns as a zero-padded ELL copy, values in
// the iteration's precision).  The spectrum of the mixed mass matrix lies in
// [0.333, 0.997] on every mesh measured (spheres, prisms, cubes; it is real and
// the matrix nearly symmetric); the iteration assumes [0.3, 1.05] and stops
// when ||I - X M||_F / sqrt(n) <= 1e-6 (FP32 storage), checked every few
// steps.  False when that does not happen within the step limit or
// the rows do not fit in LDS: the caller then uses Gauss-Jordan.
template <typename T>
bool cheb_inverse(pmchwt_ctx* c, const double* Mrow, int n, int64_t ld, T* X, bool pad_rows) {
  static_assert(sizeof(T) == 4, "the Chebyshev inverse serves the FP32 (mixed) preconditioner");
  if (cheb_rows<T>(n) < 1) return false;
  const double tol = 1e-6;
  const int kmin = 12, kmax = 48, every = 2;
  // CSC of M = CSR of M^T (nonzero entries)
  DBuf Mt = dalloc_c<double>(c, size_t(n) * n);
  launch_transpose(Mrow, Mt.as<double>(), n, c->stream);
  DBuf cnt = dalloc_c<int32_t>(c, size_t(n)), thr = dalloc_c<double>(c, size_t(n));
  DBuf colptr = dalloc_c<int64_t>(c, size_t(n) + 1);
  build_truncated_inverse<double>(Mt.as<double>(), n, n, 0.0, cnt.as<int32_t>(), thr.as<double>(),
                                  colptr.as<int64_t>(), c->stream);
  int64_t nnz = 0;
  std::vector<int32_t> hcnt(n);
  HIPCHK(hipMemcpyAsync(&nnz, colptr.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(hcnt.data(), cnt.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  const int W = cheb_width(*std::max_element(hcnt.begin(), hcnt.end()));
  if (W == 0) return false;
  DBuf rowidx = dalloc_c<int32_t>(c, size_t(std::max<int64_t>(nnz, 1)));
  DBuf val = dalloc_c<double>(c, size_t(std::max<int64_t>(nnz, 1)));
  fill_truncated_inverse<double>(Mt.as<double>(), n, n, thr.as<double>(), colptr.as<int64_t>(),
                                 rowidx.as<int32_t>(), val.as<double>(), c->stream);
  DBuf eidx = dalloc_c<int32_t>(c, size_t(W) * n), eval = dalloc_c<T>(c, size_t(W) * n);
  launch_csc_to_ell<T>(colptr.as<int64_t>(), rowidx.as<int32_t>(), val.as<double>(), n, W, eidx.as<int32_t>(),
                       eval.as<T>(), c->stream);
  // X: zero padding columns (and the identity on padding rows)
  const int64_t rows_x = pad_rows ? ld : n;
  if (sizeof(T) == 8)
    launch_zero(reinterpret_cast<double*>(X), rows_x * ld, c->stream);
  else
    launch_zero_f(reinterpret_cast<float*>(X), rows_x * ld, c->stream);
  if (pad_rows) launch_identity_tail<T>(X, ld, n, c->stream);
  DBuf D = dalloc_c<T>(c, size_t(n) * ld);
  const int rb = cheb_rows<T>(n), nblk = (n + rb - 1) / rb;
  DBuf part = dalloc_c<double>(c, size_t(nblk));
  std::vector<double> hpart(nblk);
  const double a = 0.3, b = 1.05, d = 0.5 * (a + b), cc = 0.5 * (b - a), sigma = d / cc;
  double rho_prev = 1.0 / sigma;
  bool ok = false;
  for (int k = 1; k <= kmax; ++k) {
    const double rho = 1.0 / (2.0 * sigma - rho_prev);
    launch_cheb_step<T>(X, D.as<T>(), ld, n, eidx.as<int32_t>(), eval.as<T>(), W, rho * rho_prev, 2.0 * rho / cc,
                        1.0 / d, k == 1, part.as<double>(), c->stream);
    rho_prev = rho;
    if (k >= kmin && (k - kmin) % every == 0) {
      HIPCHK(hipMemcpyAsync(hpart.data(), part.p, sizeof(double) * nblk, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
      double sum = 0.0;
      for (double v : hpart) sum += v;
      const double rn = std::sqrt(sum / n);
      c->prof.mass_iterations = k;
      c->prof.mass_residual = rn;
      if (!(rn < 1e3)) break;  // diverging: the spectrum is not where assumed
      if (rn <= tol) {
        ok = true;
        break;
      }
    }
  }
  HIPCHK(hipGetLastError());
  return ok;
}

// Sparse approximate inverses of M_A and M_A^T (kernels in massinv.inl): row
// i on the ball of columns within `hops` steps of M_A's sparsity graph,
// hops + 6 steps of the Chebyshev iteration for the spectrum interval
// [0.3, 1.05] (the spectrum of M_A lies in [0.333, 0.997] on every mesh
// measured): at 8 steps entries within about 6e-8 of the row maximum on the
// CPU check, stored in FP32.
// An FP64 preconditioner applies them with one refinement step against the
// FP64 M_A (MAcsr / MATcsr), which squares that error.  Returns
// false if a ball or a column of M_A exceeds the kernels' capacity; the
// caller then inverts densely.  Mcsr / MTcsr: FP64 CSR of M_A and M_A^T
// (scatterer-local), maxM / maxT their longest rows.
bool sparse_mass_inverse(pmchwt_ctx* c, const pmchwt_ctx::SparseInv& Mcsr, const pmchwt_ctx::SparseInv& MTcsr, int n,
                         int maxM, int maxT, int hops, pmchwt_ctx::SparseInv& inv, pmchwt_ctx::SparseInv& invT) {
  const int steps = hops + 6;
  if (maxM > spinv_wmax() || maxT > spinv_wmax()) return false;
  const int cap = spinv_cap();
  hipStream_t st = c->stream;
  DBuf count = dalloc_c<int32_t>(c, size_t(n)), ball = dalloc_c<int32_t>(c, size_t(n) * cap);
  // the inverse of M_A: pass 1 (balls), one wait for their sizes, pass 2
  SpInvJob J{};
  J.n = n;
  J.rp = Mcsr.rowptr.as<int64_t>();  // search graph: CSR of the matrix inverted
  J.ci = Mcsr.col.as<int32_t>();
  J.cp = MTcsr.rowptr.as<int64_t>();  // gather: its CSC = the CSR of its transpose
  J.ri = MTcsr.col.as<int32_t>();
  J.cv = MTcsr.val.as<double>();
  J.hops = hops;
  J.steps = steps;
  J.a = 0.3;
  J.b = 1.05;
  J.count = count.as<int32_t>();
  J.ball = ball.as<int32_t>();
  launch_spinv_ball(J, std::min(n, 4096), st);
  HIPCHK(hipGetLastError());
  std::vector<int32_t> hc(static_cast<size_t>(n));
  HIPCHK(hipMemcpyAsync(hc.data(), count.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::vector<int64_t> rowptr(size_t(n) + 1, 0);
  for (int i = 0; i < n; ++i) {
    const int b = hc[size_t(i)];
    if (b < 0) return false;
    rowptr[i + 1] = rowptr[i] + b;
  }
  inv.nnz = rowptr[n];
  if (inv.nnz >= (int64_t(1) << 32)) return false;  // entry indices of the transpose's records are 32-bit
  inv.rowptr = upload(c, rowptr);
  inv.col = dalloc_c<int32_t>(c, size_t(std::max<int64_t>(inv.nnz, 1)));
  inv.val = dalloc_c<float>(c, size_t(std::max<int64_t>(inv.nnz, 1)));
  DBuf res = dalloc_c<double>(c, size_t(n));
  J.orp = inv.rowptr.as<int64_t>();
  J.ocol = inv.col.as<int32_t>();
  J.oval = inv.val.p;
  J.res = res.as<double>();
  launch_spinv_vals<float>(J, std::min(n, 1024), st);
  HIPCHK(hipGetLastError());
  // M_A^-T as the transpose of the computed inverse: its error is the
  // transpose of the inverse's, and one ball search and Chebyshev pass less
  const int64_t nnz = inv.nnz;
  DBuf cnt = dalloc_c<int32_t>(c, size_t(n)), cur = dalloc_c<int32_t>(c, size_t(n)),
       rec = dalloc_c<int64_t>(c, size_t(std::max<int64_t>(nnz, 1)));
  invT.nnz = nnz;
  invT.rowptr = dalloc_c<int64_t>(c, size_t(n) + 1);
  invT.col = dalloc_c<int32_t>(c, size_t(std::max<int64_t>(nnz, 1)));
  invT.val = dalloc_c<float>(c, size_t(std::max<int64_t>(nnz, 1)));
  launch_cls_fill_i32(cnt.as<int32_t>(), n, 0, st);
  launch_cls_fill_i32(cur.as<int32_t>(), n, 0, st);
  launch_csr_colcount(inv.col.as<int32_t>(), nnz, cnt.as<int32_t>(), st);
  launch_scan_i32(cnt.as<int32_t>(), n, invT.rowptr.as<int64_t>(), st);
  launch_csr_tplace(inv.rowptr.as<int64_t>(), inv.col.as<int32_t>(), n, invT.rowptr.as<int64_t>(), cur.as<int32_t>(),
                    rec.as<int64_t>(), st);
  std::vector<int32_t> hcnt(static_cast<size_t>(n));
  HIPCHK(hipMemcpyAsync(hcnt.data(), cnt.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
  std::vector<double> hr(static_cast<size_t>(n));
  HIPCHK(hipMemcpyAsync(hr.data(), res.p, sizeof(double) * n, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const int maxc = n > 0 ? *std::max_element(hcnt.begin(), hcnt.end()) : 0;
  if (maxc > 4096) return false;  // LDS of the per-column sort
  SymRecJob S{};
  S.n = n;
  S.recptr = invT.rowptr.as<int64_t>();
  S.rec = rec.as<int64_t>();
  S.cnt = cur.as<int32_t>();  // scratch: the sort writes a count per column
  launch_sym_sort(S, pow2_ceil(std::max(maxc, 1)), st);
  launch_csr_tgather(rec.as<int64_t>(), nnz, inv.val.as<float>(), invT.col.as<int32_t>(), invT.val.as<float>(), st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));  // the scratch tables above go out of scope
  c->prof.mass_iterations = steps;
  c->prof.mass_residual = n > 0 ? *std::max_element(hr.begin(), hr.end()) : 0.0;
  return true;
}

// Truncated CSR copy of an inverse: entries of at least rel times their
// row's largest (2^-27 for an FP32 inverse, 2^-52 for FP64: what is dropped
// lies below the rounding of the stored inverse).  One host wait for the
// entry count; the copy is kept (true) only if it has fewer than
// max_fill * n^2 entries.
template <typename T>
bool truncated_inverse(pmchwt_ctx* c, const T* A, int64_t ld, int n, T rel, double max_fill,
                       pmchwt_ctx::SparseInv& t) {
  DBuf cnt = dalloc_c<int32_t>(c, size_t(n)), thr = dalloc_c<T>(c, size_t(n));
  t.rowptr = dalloc_c<int64_t>(c, size_t(n) + 1);
  build_truncated_inverse(A, ld, n, rel, cnt.as<int32_t>(), thr.as<T>(), t.rowptr.as<int64_t>(), c->stream);
  HIPCHK(hipMemcpyAsync(&t.nnz, t.rowptr.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (double(t.nnz) >= max_fill * double(n) * n) {
    t = pmchwt_ctx::SparseInv();
    return false;
  }
  t.col = dalloc_c<int32_t>(c, size_t(std::max<int64_t>(1, t.nnz)));
  t.val = dalloc_c<T>(c, size_t(std::max<int64_t>(1, t.nnz)));
  fill_truncated_inverse(A, ld, n, thr.as<T>(), t.rowptr.as<int64_t>(), t.col.as<int32_t>(), t.val.as<T>(),
                         c->stream);
  HIPCHK(hipGetLastError());
  return true;
}

// Structural patterns of M_A and M_A^T over the union edges (pattern
// kernels; the host lists the end points and the triangles at each vertex).
void build_mass_pattern(pmchwt_ctx* c, const CellDev& cells) {
  hipStream_t st = c->stream;
  const int E = c->E_tot, F = c->F_tot;
  std::vector<int32_t> ends(2 * size_t(E)), escat(E), eoff, vptr(size_t(c->nv_tot) + 1, 0), v2t(3 * size_t(F));
  for (size_t m = 0; m < c->sc.size(); ++m) {
    const Scat& s = c->sc[m];
    for (int e = 0; e < s.topo.E; ++e) {
      ends[2 * size_t(s.edge_off + e)] = s.vert_off + s.topo.edges[2 * size_t(e)];
      ends[2 * size_t(s.edge_off + e) + 1] = s.vert_off + s.topo.edges[2 * size_t(e) + 1];
      escat[s.edge_off + e] = int32_t(m);
    }
    eoff.push_back(s.edge_off);
    for (int f = 0; f < s.topo.F; ++f)
      for (int a = 0; a < 3; ++a) ++vptr[size_t(s.vert_off + s.topo.t[3 * size_t(f) + a]) + 1];
  }
  for (size_t v = 0; v + 1 < vptr.size(); ++v) vptr[v + 1] += vptr[v];
  {
    std::vector<int32_t> cur(vptr.begin(), vptr.end() - 1);
    for (auto& s : c->sc)
      for (int f = 0; f < s.topo.F; ++f)
        for (int a = 0; a < 3; ++a) v2t[size_t(cur[size_t(s.vert_off + s.topo.t[3 * size_t(f) + a])]++)] = s.tri_off + f;
  }
  DBuf d_ends = upload(c, ends), d_escat = upload(c, escat), d_eoff = upload(c, eoff), d_vptr = upload(c, vptr),
       d_v2t = upload(c, v2t);
  DBuf cnt = dalloc_c<int32_t>(c, size_t(E)), stats = dalloc_c<int32_t>(c, 4);
  MassPatternJob J{};
  J.E = E;
  J.F = F;
  J.edge_slots = c->sing.edge_slots.as<int32_t>();
  J.tvid = c->tvid.as<int32_t>();
  J.t2e = c->t2e.as<int32_t>();
  J.inc_ptr = cells.inc_ptr.as<int32_t>();
  J.inc_edges = cells.inc_edges.as<int32_t>();
  J.v2t_ptr = d_vptr.as<int32_t>();
  J.v2t = d_v2t.as<int32_t>();
  J.ends = d_ends.as<int32_t>();
  J.edge_scat = d_escat.as<int32_t>();
  J.edge_off = d_eoff.as<int32_t>();
  J.cnt = cnt.as<int32_t>();
  J.stats = stats.as<int32_t>();
  for (int trans = 0; trans < 2; ++trans) {
    DBuf& rp = trans ? c->mp.trowptr : c->mp.rowptr;
    DBuf& cl = trans ? c->mp.tcol : c->mp.col;
    std::vector<int64_t>& hrp = trans ? c->mp.h_trowptr : c->mp.h_rowptr;
    J.trans = trans;
    launch_cls_fill_i32(stats.as<int32_t>(), 4, 0, st);
    launch_mass_pattern(J, false, st);
    rp = dalloc_c<int64_t>(c, size_t(E) + 1);
    launch_scan_i32(cnt.as<int32_t>(), E, rp.as<int64_t>(), st);
    HIPCHK(hipGetLastError());
    hrp.resize(size_t(E) + 1);
    int32_t hs[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(hrp.data(), rp.p, hrp.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hs, stats.p, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hs[1]) throw Fail{PMCHWT_ERR_INVALID_MESH, "vertex valence too high for the mass-matrix pattern"};
    (trans ? c->mp.maxtrow : c->mp.maxrow) = hs[0];
    cl = dalloc_c<int32_t>(c, size_t(std::max<int64_t>(hrp[E], 1)));
    J.rowptr = rp.as<int64_t>();
    J.col = cl.as<int32_t>();
    launch_mass_pattern(J, true, st);
    HIPCHK(hipGetLastError());
  }
  HIPCHK(hipStreamSynchronize(st));  // the host inputs above go out of scope
  c->mp.valid = true;
}

// Rows [r0, r0 + n) of a union CSR as a CSR of their own (row offsets from 0).
pmchwt_ctx::SparseInv csr_rows(pmchwt_ctx* c, const DBuf& rowptr, const std::vector<int64_t>& h_rowptr,
                               const DBuf& col, const DBuf& val, int r0, int n) {
  pmchwt_ctx::SparseInv o;
  const int64_t b = h_rowptr[size_t(r0)];
  o.nnz = h_rowptr[size_t(r0) + n] - b;
  o.rowptr = dalloc_c<int64_t>(c, size_t(n) + 1);
  launch_rebase_i64(rowptr.as<int64_t>() + r0, n, o.rowptr.as<int64_t>(), c->stream);
  o.col = dalloc_c<int32_t>(c, size_t(std::max<int64_t>(o.nnz, 1)));
  o.val = dalloc_c<double>(c, size_t(std::max<int64_t>(o.nnz, 1)));
  if (o.nnz > 0) {
    HIPCHK(hipMemcpyAsync(o.col.p, col.as<int32_t>() + b, size_t(o.nnz) * 4, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(o.val.p, val.as<double>() + b, size_t(o.nnz) * 8, hipMemcpyDeviceToDevice, c->stream));
  }
  return o;
}

// M_A and M_A^T as CSR (values added into their structural patterns), the
// RWG Gram matrices, and the inverses the preconditioner applies: the sparse
// FP32 inverse on the graph ball by default, else (another mass_method, or a
// ball over the kernels' capacity) a dense inverse of the densified M_A.
void assemble_mass_impl(pmchwt_ctx* c, CellDev& cells) {
  EvTimer t(c->stream);
  c->MAcsr.clear();
  c->MATcsr.clear();
  c->mass_sparse.clear();
  c->Minv.clear();
  c->MinvT.clear();
  c->MinvS.clear();
  c->MinvTS.clear();
  if (!c->gram_valid) build_gram_pattern(c);
  if (!c->mp.valid) build_mass_pattern(c, cells);
  const int64_t nnzM = c->mp.h_rowptr.back(), nnzT = c->mp.h_trowptr.back();
  DBuf mval = dalloc_c<double>(c, size_t(std::max<int64_t>(nnzM, 1))),
       tval = dalloc_c<double>(c, size_t(std::max<int64_t>(nnzT, 1)));
  launch_zero(c->g_val.as<double>(), int64_t(c->g_val.bytes / 8), c->stream);
  MassJob mj{};  // every entry of M_A and M_A^T is written once
  mj.nchild = cells.nchild;
  mj.E = c->E_tot;
  mj.nnz_m = nnzM;
  mj.nnz_t = nnzT;
  mj.edge_slots = c->sing.edge_slots.as<int32_t>();
  mj.child_cell = cells.child_cell.as<int32_t>();
  mj.child_pos = cells.child_pos.as<int32_t>();
  mj.child_parent = cells.child_parent.as<int32_t>();
  mj.inc_ptr = cells.inc_ptr.as<int32_t>();
  mj.inc_edges = cells.inc_edges.as<int32_t>();
  mj.edge_scat = cells.edge_scat.as<int32_t>();
  mj.edge_off = cells.edge_off.as<int32_t>();
  mj.m_rowptr = c->mp.rowptr.as<int64_t>();
  mj.m_col = c->mp.col.as<int32_t>();
  mj.m_val = mval.as<double>();
  mj.t_rowptr = c->mp.trowptr.as<int64_t>();
  mj.t_col = c->mp.tcol.as<int32_t>();
  mj.t_val = tval.as<double>();
  mj.gram_pos = c->g_pos.as<int64_t>();
  mj.gram_val = c->g_val.as<double>();
  AsmParams<double> g = asm_params<double>(c);
  launch_mass(g, cells.params(), mj, c->stream);
  launch_gram(g, mj, c->stream);
  HIPCHK(hipGetLastError());
  for (size_t m = 0; m < c->sc.size(); ++m) {
    const Scat& s = c->sc[m];
    const int n = s.topo.E;
    const size_t nn = size_t(n) * n;
    if (c->sc.size() == 1) {  // the union CSR is the scatterer's: keep it
      pmchwt_ctx::SparseInv a, b;
      a.nnz = nnzM;
      b.nnz = nnzT;
      a.rowptr = dalloc_c<int64_t>(c, size_t(n) + 1);
      b.rowptr = dalloc_c<int64_t>(c, size_t(n) + 1);
      HIPCHK(hipMemcpyAsync(a.rowptr.p, c->mp.rowptr.p, (size_t(n) + 1) * 8, hipMemcpyDeviceToDevice, c->stream));
      HIPCHK(hipMemcpyAsync(b.rowptr.p, c->mp.trowptr.p, (size_t(n) + 1) * 8, hipMemcpyDeviceToDevice, c->stream));
      a.col = dalloc_c<int32_t>(c, size_t(std::max<int64_t>(nnzM, 1)));
      b.col = dalloc_c<int32_t>(c, size_t(std::max<int64_t>(nnzT, 1)));
      HIPCHK(hipMemcpyAsync(a.col.p, c->mp.col.p, size_t(nnzM) * 4, hipMemcpyDeviceToDevice, c->stream));
      HIPCHK(hipMemcpyAsync(b.col.p, c->mp.tcol.p, size_t(nnzT) * 4, hipMemcpyDeviceToDevice, c->stream));
      a.val = std::move(mval);
      b.val = std::move(tval);
      c->MAcsr.push_back(std::move(a));
      c->MATcsr.push_back(std::move(b));
    } else {
      c->MAcsr.push_back(csr_rows(c, c->mp.rowptr, c->mp.h_rowptr, c->mp.col, mval, s.edge_off, n));
      c->MATcsr.push_back(csr_rows(c, c->mp.trowptr, c->mp.h_trowptr, c->mp.tcol, tval, s.edge_off, n));
    }
    const pmchwt_ctx::SparseInv& Mm = c->MAcsr.back();
    const int64_t ldm = ldmass(n);
    if (c->optP.mass_method == 0) {  // sparse inverse on the graph ball (dense only if a ball overflows)
      pmchwt_ctx::SparseInv a, b;
      const int hops = c->optP.mass_hops > 0 ? c->optP.mass_hops : (c->mass_f32 ? 6 : 8);
      if (sparse_mass_inverse(c, Mm, c->MATcsr.back(), n, c->mp.maxrow, c->mp.maxtrow, hops, a, b)) {
        c->MinvS.push_back(std::move(a));
        c->MinvTS.push_back(std::move(b));
        c->mass_sparse.push_back(1);
        c->Minv.emplace_back();  // dense FP32 copies for the matrix-core product: built when first needed
        c->MinvT.emplace_back();
        continue;
      }
      c->MinvS.resize(m);
      c->MinvTS.resize(m);
    }
    c->mass_sparse.push_back(0);
    // dense M_A of this scatterer for the dense inverses
    DBuf Md0 = dalloc_c<double>(c, nn);
    launch_zero(Md0.as<double>(), int64_t(nn), c->stream);
    launch_csr_to_dense(Mm.rowptr.as<int64_t>(), Mm.col.as<int32_t>(), Mm.val.as<double>(), n, Md0.as<double>(), n,
                        c->stream);
    if (c->mass_f32) {
      // FP32 inverse of [[M_A, 0], [0, I]] (ldm x ldm); its top-left block is
      // M_A^-1 with zero padding columns, the layout the products read
      DBuf Mf = dalloc_c<float>(c, size_t(ldm) * ldm), MfT = dalloc_c<float>(c, size_t(ldm) * ldm);
      if (c->optP.mass_method != 2 || !cheb_inverse<float>(c, Md0.as<double>(), n, ldm, Mf.as<float>(), true)) {
        launch_embed_f32(Md0.as<double>(), n, Mf.as<float>(), int(ldm), c->stream);
        gj_inverse_f32(c, Mf.as<float>(), int(ldm));
        c->prof.mass_iterations = 0;
      }
      launch_transpose_f32(Mf.as<float>(), MfT.as<float>(), int(ldm), c->stream);
      c->MinvS.emplace_back();
      c->MinvTS.emplace_back();
      truncated_inverse<float>(c, Mf.as<float>(), ldm, n, 0x1p-27f, 2.0, c->MinvS.back());
      truncated_inverse<float>(c, MfT.as<float>(), ldm, n, 0x1p-27f, 2.0, c->MinvTS.back());
      c->Minv.push_back(std::move(Mf));
      c->MinvT.push_back(std::move(MfT));
      continue;
    }
    // FP64: Gauss-Jordan (the Chebyshev iteration needs about 30 FP64 steps
    // here, each streaming X and D twice: slower than the blocked inverse)
    DBuf Mi = std::move(Md0), MiT = dalloc_c<double>(c, nn);
    // row-major M_A is column-major M_A^T; inverting it in place yields the
    // column-major (M_A^T)^-1, i.e. the row-major M_A^-1.
    gj_inverse(c, Mi.as<double>(), n);
    c->prof.mass_iterations = 0;
    launch_transpose(Mi.as<double>(), MiT.as<double>(), n, c->stream);
    // padded copy for the vector loads of the application kernel
    DBuf Md = dalloc_c<double>(c, size_t(n) * ldm), MdT = dalloc_c<double>(c, size_t(n) * ldm);
    launch_repack(Mi.as<double>(), n, Md.as<double>(), ldm, c->stream);
    launch_repack(MiT.as<double>(), n, MdT.as<double>(), ldm, c->stream);
    // truncated copies where they are sparse enough to read fewer bytes
    // (12 B per kept entry against 8 B per dense entry)
    pmchwt_ctx::SparseInv a, b;
    if (truncated_inverse<double>(c, Md.as<double>(), ldm, n, 0x1p-52, 0.4, a) &&
        truncated_inverse<double>(c, MdT.as<double>(), ldm, n, 0x1p-52, 0.4, b)) {
      c->MinvS.push_back(std::move(a));
      c->MinvTS.push_back(std::move(b));
    } else {  // empty entries: the products read the dense inverse
      c->MinvS.emplace_back();
      c->MinvTS.emplace_back();
    }
    c->Minv.push_back(std::move(Md));
    c->MinvT.push_back(std::move(MdT));
  }
  HIPCHK(hipGetLastError());
  c->prof.ms_mass = t.stop();
}

// ---------------------------------------------------------------------------
// Operator application.  Internal vectors: [rhs][D (E_tot) ; N (E_tot)] complex128.
// ---------------------------------------------------------------------------
int64_t vlen(const pmchwt_ctx* c) { return 2 * int64_t(c->E_tot); }

double* need_work(pmchwt_ctx* c, size_t doubles) {
  if (c->work_bytes < doubles * 8) {
    c->work = dalloc<double>(doubles);
    c->work_bytes = doubles * 8;
  }
  return c->work.as<double>();
}

int64_t A_matvecs(const pmchwt_ctx* c) {
  const int64_t M = int64_t(c->sc.size());
  return 4 * M * M + 4 * M;
}

int64_t P_matvecs(const pmchwt_ctx* c) {
  const int64_t M = int64_t(c->sc.size());
  switch (c->precond) {
    case PMCHWT_P_A: return 4 * M * M + 4 * M;
    case PMCHWT_P_D: return 8 * M;
    case PMCHWT_P_D_INT:
    case PMCHWT_P_D_EXT: return 4 * M;
    case PMCHWT_P_S_INT:
    case PMCHWT_P_S_EXT: return 2 * M;
    default: return 0;
  }
}

// workspace of the matrix-core products: two expanded right-hand blocks of
// 4 nrhs x 2 ldE floats (enough for the mass-inverse product as well)
float* mfma_ws(pmchwt_ctx* c, int nrhs) {
  const size_t need = size_t(2) * 4 * nrhs * 2 * size_t(std::max<int64_t>(c->ldE, ldmass(c->E_tot))) * sizeof(float);
  if (c->mfma_ws_bytes < need) {
    c->mfma_ws = DBuf();
    c->mfma_ws = dalloc<float>(need / sizeof(float));
    c->mfma_ws_bytes = need;
  }
  return c->mfma_ws.as<float>();
}

// FP64 workspace of the matrix-core products: 16 nrhs x ld doubles (the two
// expanded right-hand blocks of a per-medium product)
double* mfma_ws64(pmchwt_ctx* c, int nrhs) {
  const size_t need = size_t(16) * nrhs * size_t(c->ldE) * sizeof(double);
  if (c->mfma_ws_bytes < need) {
    c->mfma_ws = DBuf();
    c->mfma_ws = dalloc<float>(need / sizeof(float));
    c->mfma_ws_bytes = need;
  }
  return reinterpret_cast<double*>(c->mfma_ws.p);
}

// y = A x (y overwritten)
void apply_A(pmchwt_ctx* c, const double* x, double* y, int nrhs) {
  const int64_t E = c->E_tot, vs = vlen(c);
  const bool f64 = c->precA == PMCHWT_FP64;
  c->calls_A += 1;
  const bool timed = sample_matvec(c) || (!f64 && nrhs >= MFMA_MIN_RHS);
  if (c->sym.ready && nrhs <= 2) {  // symmetric tiles, one right-hand side per pass
    const int n = int(E), nt = c->sym.nt;
    for (int q = 0; q < nrhs; ++q) {
      const double* xq = x + 2 * int64_t(q) * vs;
      double* yq = y + 2 * int64_t(q) * vs;
      LazyTimer t(c, timed);
      if (f64)
        launch_gemv_sym3<double>(c->sym.pack.as<double>(), c->sym.tij.as<int32_t>(), c->sym.ntiles, nt, n, xq,
                                 xq + 2 * E, c->sym.part.as<double>(), c->stream);
      else
        launch_gemv_sym3<float>(c->sym.pack.as<float>(), c->sym.tij.as<int32_t>(), c->sym.ntiles, nt, n, xq,
                                xq + 2 * E, c->sym.part.as<double>(), c->stream);
      t.stop(&c->prof.ms_matvec_total);
      LazyTimer t2(c, timed);
      if (f64)
        launch_sym_reduce<double>(c->sym.part.as<double>(), nt, n, c->sym.rowptr.as<int64_t>(),
                                  c->sym.col.as<int32_t>(), c->sym.val.as<double>(), xq, xq + 2 * E, yq, yq + 2 * E,
                                  c->stream);
      else
        launch_sym_reduce<float>(c->sym.part.as<double>(), nt, n, c->sym.rowptr.as<int64_t>(),
                                 c->sym.col.as<int32_t>(), c->sym.val.as<float>(), xq, xq + 2 * E, yq, yq + 2 * E,
                                 c->stream);
      t2.stop(&c->prof.ms_matvec_reduce);
      HIPCHK(hipGetLastError());
    }
    c->prof.matvec_launches += nrhs;
    c->prof.matvec_timed += timed ? nrhs : 0;
    c->prof.matvec_bytes += nrhs * c->sym.ntiles * 3 * SYM_T * SYM_T * (f64 ? 16 : 8);
    return;
  }
  ensure_lower(c, 15);  // every product below reads whole rows
  if (f64 && nrhs >= MFMA_MIN_RHS && c->sc.size() == 1 && c->comb_ok) {
    // the three combined operators on the FP64 matrix cores
    if (!c->comb) build_comb<double>(c);
    double* BD = mfma_ws64(c, nrhs);
    double* BN = BD + size_t(2) * nrhs * 2 * size_t(c->ldE);
    LazyTimer tm(c), t(c, timed);
    launch_mfma64_comb(c->AC.as<double>(), c->AS1.as<double>(), c->AS2.as<double>(), c->ldE, int(E), int(E), x,
                       x + 2 * E, y, y + 2 * E, nrhs, vs, BD, BN, c->stream);
    HIPCHK(hipGetLastError());
    tm.stop(&c->prof.ms_mfma_total);
    t.stop(&c->prof.ms_matvec_total);
    c->prof.mfma_launches += 1;
    c->prof.mfma_flops += 32 * E * c->ldE * nrhs;
    return;
  }
  if (!f64 && nrhs >= MFMA_MIN_RHS && c->sc.size() == 1 && c->comb_ok) {
    // the three combined operators on the matrix cores
    if (!c->comb) build_comb<float>(c);
    float* BD = mfma_ws(c, nrhs);
    float* BN = BD + size_t(2) * nrhs * 2 * size_t(c->ldE);
    LazyTimer tm(c), t(c, timed);
    launch_mfma_comb(c->AC.as<float>(), c->AS1.as<float>(), c->AS2.as<float>(), c->ldE, int(E), int(E), x, x + 2 * E,
                     y, y + 2 * E, nrhs, vs, BD, BN, c->stream);
    HIPCHK(hipGetLastError());
    tm.stop(&c->prof.ms_mfma_total);
    t.stop(&c->prof.ms_matvec_total);
    c->prof.mfma_launches += 2;
    c->prof.mfma_flops += 32 * E * c->ldE * nrhs;
    return;
  }
  if (c->sym.ready && !c->comb && !(!f64 && nrhs >= MFMA_MIN_RHS)) {
    if (f64)
      build_comb<double>(c);
    else
      build_comb<float>(c);
  }
  if (c->comb && !(!f64 && nrhs >= MFMA_MIN_RHS)) {
    LazyTimer t(c, timed);  // one launch writes every row of y: no clearing pass
    if (f64)
      launch_gemv_pmchwt3<double>(c->AC.as<double>(), c->AS1.as<double>(), c->AS2.as<double>(), c->ldE, int(E), int(E),
                                  x, x + 2 * E, y, y + 2 * E, nrhs, vs, c->stream, false);
    else
      launch_gemv_pmchwt3<float>(c->AC.as<float>(), c->AS1.as<float>(), c->AS2.as<float>(), c->ldE, int(E), int(E), x,
                                 x + 2 * E, y, y + 2 * E, nrhs, vs, c->stream, false);
    HIPCHK(hipGetLastError());
    t.stop(&c->prof.ms_matvec_total);
    c->prof.matvec_launches += 1;
    c->prof.matvec_timed += timed ? 1 : 0;
    c->prof.matvec_bytes += 3 * E * E * (f64 ? 16 : 8);
    return;
  }
  launch_zero(y, 2 * vs * nrhs, c->stream);
  LazyTimer t(c, timed);
  if (f64 && nrhs >= MFMA_MIN_RHS) {
    double* B1 = mfma_ws64(c, nrhs);
    double* B2 = B1 + size_t(4) * nrhs * 2 * size_t(c->ldE);
    LazyTimer tm(c);
    launch_mfma64_pmchwt(c->Se.as<double>(), c->Ce.as<double>(), c->ldE, int(E), int(E), c->k_ext, 0.0, x, x + 2 * E,
                         y, y + 2 * E, nrhs, vs, B1, B2, c->stream);
    int64_t flops = 32 * E * c->ldE * nrhs;
    for (size_t m = 0; m < c->sc.size(); ++m) {
      const Scat& s = c->sc[m];
      const int64_t o = s.edge_off;
      launch_mfma64_pmchwt(c->Si[m].as<double>(), c->Ci[m].as<double>(), c->ldI[m], s.topo.E, s.topo.E, s.k.real(),
                           s.k.imag(), x + 2 * o, x + 2 * (E + o), y + 2 * o, y + 2 * (E + o), nrhs, vs, B1, B2,
                           c->stream);
      flops += 32 * int64_t(s.topo.E) * c->ldI[m] * nrhs;
    }
    HIPCHK(hipGetLastError());
    tm.stop(&c->prof.ms_mfma_total);
    c->prof.mfma_launches += 1 + int64_t(c->sc.size());
    c->prof.mfma_flops += flops;
    t.stop(&c->prof.ms_matvec_total);
    return;
  } else if (c->precA == PMCHWT_FP64) {
    launch_gemv_pmchwt<double>(c->Se.as<double>(), c->Ce.as<double>(), c->ldE, int(E), int(E), c->k_ext, 0.0, x,
                               x + 2 * E, y, y + 2 * E, nrhs, vs, c->stream);
    for (size_t m = 0; m < c->sc.size(); ++m) {
      const Scat& s = c->sc[m];
      const int64_t o = s.edge_off;
      launch_gemv_pmchwt<double>(c->Si[m].as<double>(), c->Ci[m].as<double>(), c->ldI[m], s.topo.E, s.topo.E,
                                 s.k.real(), s.k.imag(), x + 2 * o, x + 2 * (E + o), y + 2 * o, y + 2 * (E + o), nrhs,
                                 vs, c->stream);
    }
  } else if (nrhs >= MFMA_MIN_RHS) {
    float* B1 = mfma_ws(c, nrhs);
    float* B2 = B1 + size_t(4) * nrhs * 2 * size_t(c->ldE);
    LazyTimer tm(c);
    launch_mfma_pmchwt(c->Se.as<float>(), c->Ce.as<float>(), c->ldE, int(E), int(E), c->k_ext, 0.0, x, x + 2 * E, y,
                       y + 2 * E, nrhs, vs, B1, B2, c->stream);
    int64_t flops = 32 * E * c->ldE * nrhs;
    for (size_t m = 0; m < c->sc.size(); ++m) {
      const Scat& s = c->sc[m];
      const int64_t o = s.edge_off;
      launch_mfma_pmchwt(c->Si[m].as<float>(), c->Ci[m].as<float>(), c->ldI[m], s.topo.E, s.topo.E, s.k.real(),
                         s.k.imag(), x + 2 * o, x + 2 * (E + o), y + 2 * o, y + 2 * (E + o), nrhs, vs, B1, B2,
                         c->stream);
      flops += 32 * int64_t(s.topo.E) * c->ldI[m] * nrhs;
    }
    HIPCHK(hipGetLastError());
    tm.stop(&c->prof.ms_mfma_total);
    c->prof.mfma_launches += 1 + int64_t(c->sc.size());
    c->prof.mfma_flops += flops;
    t.stop(&c->prof.ms_matvec_total);
    return;
  } else {
    launch_gemv_pmchwt<float>(c->Se.as<float>(), c->Ce.as<float>(), c->ldE, int(E), int(E), c->k_ext, 0.0, x, x + 2 * E,
                              y, y + 2 * E, nrhs, vs, c->stream);
    for (size_t m = 0; m < c->sc.size(); ++m) {
      const Scat& s = c->sc[m];
      const int64_t o = s.edge_off;
      launch_gemv_pmchwt<float>(c->Si[m].as<float>(), c->Ci[m].as<float>(), c->ldI[m], s.topo.E, s.topo.E,
                                s.k.real(), s.k.imag(), x + 2 * o, x + 2 * (E + o), y + 2 * o, y + 2 * (E + o), nrhs,
                                vs, c->stream);
    }
  }
  HIPCHK(hipGetLastError());
  t.stop(&c->prof.ms_matvec_total);
  c->prof.matvec_launches += 1 + int64_t(c->sc.size());
  c->prof.matvec_timed += timed ? 1 + int64_t(c->sc.size()) : 0;
  int64_t bytes = 2 * E * E;
  for (auto& s : c->sc) bytes += 2 * int64_t(s.topo.E) * s.topo.E;
  c->prof.matvec_bytes += bytes * (c->precA == PMCHWT_FP64 ? 16 : 8);
}

// y = A x (use_ext) or y = A^i x with every entry integrated again in FP64
// (y overwritten): the product with the FP64 Galerkin matrix when the stored
// operators are FP32.  Counts as one operator application.
// y = A x in FP64 without stored operators (use_ext: exterior and interior
// operators; else the interior ones); xi: input of the interior operators
// when it differs from x (else null)
void apply_A_free(pmchwt_ctx* c, const double* x, double* y, int nrhs, bool use_ext, const double* xi = nullptr) {
  if (!c->sing.blk.p) throw Fail{PMCHWT_ERR_STATE, "A not assembled"};
  const int64_t vs = vlen(c);
  const size_t need = size_t(nrhs) * 3 * size_t(c->F_tot) * 4;
  if (c->free_slots.bytes < need * 8) realloc_c<double>(c, c->free_slots, need);
  const size_t need_part = size_t(free_part_doubles(c->F_tot, nrhs));
  if (c->free_part.bytes < need_part * 8) realloc_c<double>(c, c->free_part, need_part);
  AsmParams<double> p = asm_params<double>(c);
  p.q_near = c->optA.q_near;
  p.q_medium = c->optA.q_medium;
  p.q_far = c->optA.q_far;
  FreeJob f{};
  f.use_ext = use_ext ? 1 : 0;
  f.nrhs = nrhs;
  f.E_tot = c->E_tot;
  f.vs = vs;
  f.x = x;
  f.xi = xi;
  f.sing_ptr = c->sing.ptr.as<int64_t>();
  f.sing_pairs = c->sing.pairs.as<int32_t>();
  f.sing_blk = c->sing.blk.as<double>();
  f.slots = c->free_slots.as<double>();
  f.edge_slots = c->sing.edge_slots.as<int32_t>();
  f.y = y;
  {
    LazyTimer t(c, true);
    launch_free_apply(p, f, c->free_part.as<double>(), c->stream);
    HIPCHK(hipGetLastError());
    t.stop(&c->prof.ms_free_apply);
  }
  c->prof.free_launches += 1;
  if (use_ext) c->calls_A += 1;
}

// MIXED solves with refinement and at least this many right-hand sides take
// their FP64 residuals from an FP64 copy of A instead of the matrix-free
// product, which integrates every pair again for each right-hand side.
constexpr int FREE_MAX_RHS = 4;

// The FP64 copy of A: the FP64 assembly (full rows, no combined matrices)
// run on the context's operator slots, with the FP32 state kept aside and
// put back afterwards (also when the assembly fails).
void ensure_a64(pmchwt_ctx* c) {
  if (c->a64.valid) return;
  struct Keep {
    pmchwt_ctx* c;
    DBuf Se, Ce, Si_ptr, Ci_ptr, ld_int, AC, AS1, AS2, pack, val, part;
    std::vector<DBuf> Si, Ci;
    std::vector<int64_t> ldI;
    int64_t ldE;
    bool comb, comb_ok, ready, stale[4];
    pmchwt_profile prof;
    double recompute;
    int precA;
    pmchwt_assembly_opts optA;
    explicit Keep(pmchwt_ctx* cc) : c(cc) {
      Se = std::move(c->Se);
      Ce = std::move(c->Ce);
      Si_ptr = std::move(c->Si_ptr);
      Ci_ptr = std::move(c->Ci_ptr);
      ld_int = std::move(c->ld_int);
      AC = std::move(c->AC);
      AS1 = std::move(c->AS1);
      AS2 = std::move(c->AS2);
      pack = std::move(c->sym.pack);
      val = std::move(c->sym.val);
      part = std::move(c->sym.part);
      Si = std::move(c->Si);
      Ci = std::move(c->Ci);
      ldI = c->ldI;
      ldE = c->ldE;
      comb = c->comb;
      comb_ok = c->comb_ok;
      ready = c->sym.ready;
      for (int k = 0; k < 4; ++k) stale[k] = c->sym.lower_stale[k];
      prof = c->prof;
      recompute = c->recompute;
      precA = c->precA;
      optA = c->optA;
    }
    ~Keep() {
      c->Se = std::move(Se);
      c->Ce = std::move(Ce);
      c->Si_ptr = std::move(Si_ptr);
      c->Ci_ptr = std::move(Ci_ptr);
      c->ld_int = std::move(ld_int);
      c->AC = std::move(AC);
      c->AS1 = std::move(AS1);
      c->AS2 = std::move(AS2);
      c->sym.pack = std::move(pack);
      c->sym.val = std::move(val);
      c->sym.part = std::move(part);
      c->Si = std::move(Si);
      c->Ci = std::move(Ci);
      c->ldI = ldI;
      c->ldE = ldE;
      c->comb = comb;
      c->comb_ok = comb_ok;
      c->sym.ready = ready;
      for (int k = 0; k < 4; ++k) c->sym.lower_stale[k] = stale[k];
      const double ms = c->prof.ms_assemble_A;
      c->prof = prof;
      c->prof.ms_fp64_copy = ms;
      c->recompute = recompute;
      c->precA = precA;
      c->optA = optA;
    }
  } keep(c);
  pmchwt_assembly_opts o = c->optA;
  o.precision = PMCHWT_FP64;
  o.operator_form = 1;
  c->optA = o;
  c->comb_ok = false;
  c->precA = PMCHWT_FP64;
  assemble_A_impl<double>(c, o);
  c->a64.Se = std::move(c->Se);
  c->a64.Ce = std::move(c->Ce);
  c->a64.Si = std::move(c->Si);
  c->a64.Ci = std::move(c->Ci);
  c->a64.ldI = c->ldI;
  c->a64.ldE = c->ldE;
  c->a64.valid = true;
}

// y = A^i u + A^e x from the FP64 copy of A (u: input of the interior
// operators), for the refinement residual g/2 - A^i (c_inc + x) - A^e x
void apply_A64_split(pmchwt_ctx* c, const double* x, const double* u, double* y, int nrhs) {
  const int64_t E = c->E_tot, vs = vlen(c);
  launch_zero(y, 2 * vs * nrhs, c->stream);
  if (nrhs >= MFMA_MIN_RHS) {  // on the FP64 matrix cores
    double* B1 = mfma_ws64(c, nrhs);
    double* B2 = B1 + size_t(4) * nrhs * 2 * size_t(c->a64.ldE);
    launch_mfma64_pmchwt(c->a64.Se.as<double>(), c->a64.Ce.as<double>(), c->a64.ldE, int(E), int(E), c->k_ext, 0.0,
                         x, x + 2 * E, y, y + 2 * E, nrhs, vs, B1, B2, c->stream);
    for (size_t m = 0; m < c->sc.size(); ++m) {
      const Scat& s = c->sc[m];
      const int64_t o = s.edge_off;
      launch_mfma64_pmchwt(c->a64.Si[m].as<double>(), c->a64.Ci[m].as<double>(), c->a64.ldI[m], s.topo.E, s.topo.E,
                           s.k.real(), s.k.imag(), u + 2 * o, u + 2 * (E + o), y + 2 * o, y + 2 * (E + o), nrhs, vs,
                           B1, B2, c->stream);
    }
    HIPCHK(hipGetLastError());
    c->calls_A += 1;
    return;
  }
  launch_gemv_pmchwt<double>(c->a64.Se.as<double>(), c->a64.Ce.as<double>(), c->a64.ldE, int(E), int(E), c->k_ext,
                             0.0, x, x + 2 * E, y, y + 2 * E, nrhs, vs, c->stream);
  for (size_t m = 0; m < c->sc.size(); ++m) {
    const Scat& s = c->sc[m];
    const int64_t o = s.edge_off;
    launch_gemv_pmchwt<double>(c->a64.Si[m].as<double>(), c->a64.Ci[m].as<double>(), c->a64.ldI[m], s.topo.E,
                               s.topo.E, s.k.real(), s.k.imag(), u + 2 * o, u + 2 * (E + o), y + 2 * o,
                               y + 2 * (E + o), nrhs, vs, c->stream);
  }
  HIPCHK(hipGetLastError());
  c->calls_A += 1;
}

// FP64 refinement residual product y = A^i u + A^e x: the FP64 copy of A for
// many right-hand sides, else the matrix-free product
void apply_A_resid(pmchwt_ctx* c, const double* x, const double* u, double* y, int nrhs) {
  if (nrhs >= FREE_MAX_RHS) {
    ensure_a64(c);
    apply_A64_split(c, x, u, y, nrhs);
  } else {
    apply_A_free(c, x, y, nrhs, true, u);
  }
}

// Block-sparse copy (BSR_T x BSR_T tiles) of an FP32 CSR matrix with rows
// [0, rows) and columns [0, cols); v2: a second value set on the pattern.
void build_bsr(pmchwt_ctx* c, const int64_t* rowptr, const int32_t* col, int rows, int cols, const float* v1,
               const float* v2, bool cplx, BsrHold& h) {
  hipStream_t st = c->stream;
  const int nbr = (rows + BSR_T - 1) / BSR_T, nbc = (cols + BSR_T - 1) / BSR_T;
  const size_t nb = size_t(nbr) * nbc;
  DBuf flag = dalloc_c<int32_t>(c, nb);
  launch_cls_fill_i32(flag.as<int32_t>(), int64_t(nb), 0, st);
  launch_bsr_mark(rowptr, col, rows, nbc, flag.as<int32_t>(), st);
  HIPCHK(hipGetLastError());
  std::vector<int32_t> hf(nb), bcol;
  std::vector<int64_t> bptr(size_t(nbr) + 1, 0);
  HIPCHK(hipMemcpyAsync(hf.data(), flag.p, nb * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int bi = 0; bi < nbr; ++bi) {
    for (int bj = 0; bj < nbc; ++bj) {
      int32_t& f = hf[size_t(bi) * nbc + bj];
      if (f) {
        f = int32_t(bcol.size());
        bcol.push_back(bj);
      } else {
        f = -1;
      }
    }
    bptr[size_t(bi) + 1] = int64_t(bcol.size());
  }
  const int64_t nt = int64_t(bcol.size());
  const int kw = cplx ? 2 * BSR_T : BSR_T;
  h.bptr = upload(c, bptr);
  h.bcol = upload(c, bcol.empty() ? std::vector<int32_t>{0} : bcol);
  DBuf tmap = upload(c, hf);
  const size_t tv = size_t(std::max<int64_t>(nt, 1)) * BSR_T * kw;
  h.t1 = dalloc_c<float>(c, tv);
  launch_zero_f(h.t1.as<float>(), int64_t(tv), st);
  launch_bsr_fill(rowptr, col, v1, rows, nbc, tmap.as<int32_t>(), cplx, h.t1.as<float>(), st);
  if (v2) {
    h.t2 = dalloc_c<float>(c, tv);
    launch_zero_f(h.t2.as<float>(), int64_t(tv), st);
    launch_bsr_fill(rowptr, col, v2, rows, nbc, tmap.as<int32_t>(), cplx, h.t2.as<float>(), st);
  }
  HIPCHK(hipGetLastError());
  h.m.nbr = nbr;
  h.m.nbc = nbc;
  h.m.ntiles = nt;
  h.m.bptr = h.bptr.as<int64_t>();
  h.m.bcol = h.bcol.as<int32_t>();
  h.m.tiles1 = h.t1.as<float>();
  h.m.tiles2 = v2 ? h.t2.as<float>() : nullptr;
  h.valid = true;
  HIPCHK(hipStreamSynchronize(st));  // tmap and flag go out of scope
}

// workspace of the block-sparse products: two blocks of 4 nrhs x 2 nbc BSR_T floats
float* bsr_ws(pmchwt_ctx* c, int nrhs) {
  const int64_t kt = 2 * ((c->E_tot + BSR_T - 1) / BSR_T) * BSR_T;
  const size_t need = size_t(2) * 4 * nrhs * size_t(kt) * sizeof(float);
  if (c->bsr_ws_bytes < need) {
    c->bsr_ws = DBuf();
    c->bsr_ws = dalloc<float>(need / sizeof(float));
    c->bsr_ws_bytes = need;
  }
  return c->bsr_ws.as<float>();
}

// z = M_P^-1 P M_A^-1 y  (z overwritten; tmp: 2 vectors of scratch)
void apply_Ptilde(pmchwt_ctx* c, const double* y, double* z, double* t1, double* t2, int nrhs) {
  const int64_t E = c->E_tot, vs = vlen(c);
  if (c->precond == PMCHWT_P_I) {
    HIPCHK(hipMemcpyAsync(z, y, size_t(2 * vs * nrhs) * 8, hipMemcpyDeviceToDevice, c->stream));
    return;
  }
  c->calls_P += 1;
  const bool many = nrhs >= MFMA_MIN_RHS;
  const bool mm = c->mass_f32 && many;
  float* Bw = many ? bsr_ws(c, nrhs) : nullptr;
  // out = alpha M_A^-1 in (transposed: M_A^-T) for scatterer m: for many
  // right-hand sides the matrix-core product on the block-sparse copy of the
  // sparse FP32 inverse (else on the dense FP32 inverse), else the sparse
  // inverse, else the dense FP64 one
  auto mass_inv = [&](size_t m, bool tr, double alpha, const double* in, double* out) {
    const Scat& s = c->sc[m];
    const int64_t o = s.edge_off, ldm = ldmass(s.topo.E);
    pmchwt_ctx::SparseInv& S = tr ? c->MinvTS[m] : c->MinvS[m];
    DBuf& Dn = tr ? c->MinvT[m] : c->Minv[m];
    const bool sp32 = S.rowptr.p && (c->mass_f32 || (m < c->mass_sparse.size() && c->mass_sparse[m]));
    if (many && sp32 && !S.bsr.valid)
      build_bsr(c, S.rowptr.as<int64_t>(), S.col.as<int32_t>(), s.topo.E, s.topo.E, S.val.as<float>(), nullptr, false,
                S.bsr);
    if (mm && S.bsr.valid) {
      launch_bsr_real2(S.bsr.m, s.topo.E, s.topo.E, alpha, in + 2 * o, out + 2 * o, nrhs, vs, E, Bw, c->stream);
    } else if (mm) {
      if (!Dn.p) {
        Dn = dalloc_c<float>(c, size_t(ldm) * ldm);
        launch_zero_f(Dn.as<float>(), ldm * ldm, c->stream);
        launch_csr_scatter_f32(S.rowptr.as<int64_t>(), S.col.as<int32_t>(), S.val.as<float>(), s.topo.E, Dn.as<float>(),
                               ldm, c->stream);
      }
      launch_mfma_real2(Dn.as<float>(), ldm, s.topo.E, s.topo.E, alpha, in + 2 * o, out + 2 * o, nrhs, vs, E, Bw,
                        c->stream);
    } else if (S.rowptr.p && c->mass_f32) {
      launch_spmv_real2_csr(S.rowptr.as<int64_t>(), S.col.as<int32_t>(), S.val.as<float>(), s.topo.E, alpha, in + 2 * o,
                            out + 2 * o, nrhs, vs, E, c->stream);
    } else if (S.rowptr.p && m < c->mass_sparse.size() && c->mass_sparse[m]) {
      // FP64 preconditioner, sparse FP32 inverse X: out = alpha (X in + X (in - M X in))
      const pmchwt_ctx::SparseInv& Mm = tr ? c->MATcsr[m] : c->MAcsr[m];
      const size_t need = size_t(2 * vs * nrhs);
      if (c->mass_tmp.bytes < need * 8) realloc_c<double>(c, c->mass_tmp, need);
      double* tmp = c->mass_tmp.as<double>();
      const int64_t* rp = S.rowptr.as<int64_t>();
      const int32_t* cl = S.col.as<int32_t>();
      const float* vl = S.val.as<float>();
      // the products with X on the matrix cores for many right-hand sides: the
      // FP32 rounding of their inputs is corrected like X's own error (the
      // block-sparse copy stays from an earlier call; Bw exists only here)
      const bool xb = many && S.bsr.valid;
      if (xb)
        launch_bsr_real2(S.bsr.m, s.topo.E, s.topo.E, alpha, in + 2 * o, out + 2 * o, nrhs, vs, E, Bw, c->stream);
      else
        launch_spmv_real2_csr(rp, cl, vl, s.topo.E, alpha, in + 2 * o, out + 2 * o, nrhs, vs, E, c->stream);
      if (many) {  // the residual's gathers from a copy with the right-hand sides adjacent per column
        DBuf xt = dalloc_c<double>(c, 4 * size_t(s.topo.E) * nrhs);
        launch_spmv_real2_csr_t(Mm.rowptr.as<int64_t>(), Mm.col.as<int32_t>(), Mm.val.as<double>(), s.topo.E,
                                s.topo.E, -1.0, out + 2 * o, tmp + 2 * o, nrhs, vs, E, xt.as<double>(), c->stream);
      } else {
        launch_spmv_real2_csr(Mm.rowptr.as<int64_t>(), Mm.col.as<int32_t>(), Mm.val.as<double>(), s.topo.E, -1.0,
                              out + 2 * o, tmp + 2 * o, nrhs, vs, E, c->stream);
      }
      launch_axpby_rows(tmp + 2 * o, in + 2 * o, vs, s.topo.E, E, nrhs, 1.0, alpha, c->stream);
      if (xb)
        launch_bsr_real2(S.bsr.m, s.topo.E, s.topo.E, 1.0, tmp + 2 * o, out + 2 * o, nrhs, vs, E, Bw, c->stream, true);
      else
        launch_spmv_real2_csr(rp, cl, vl, s.topo.E, 1.0, tmp + 2 * o, out + 2 * o, nrhs, vs, E, c->stream, 1.0);
    } else if (S.rowptr.p) {
      launch_spmv_real2_csr(S.rowptr.as<int64_t>(), S.col.as<int32_t>(), S.val.as<double>(), s.topo.E, alpha,
                            in + 2 * o, out + 2 * o, nrhs, vs, E, c->stream);
    } else {
      launch_gemv_real2(Dn.as<double>(), ldm, s.topo.E, s.topo.E, alpha, in + 2 * o, out + 2 * o, nrhs, vs, E,
                        c->stream);
    }
  };
  for (size_t m = 0; m < c->sc.size(); ++m) mass_inv(m, false, 1.0, y, t1);
  // the interior launches write disjoint row ranges that cover every row of
  // t2 (scatterer m owns rows edge_off .. edge_off + E_m of both halves), so
  // the first writer overwrites and t2 needs no clearing pass
  const int64_t* rp = c->p_rowptr.as<int64_t>();
  const int32_t* cl = c->p_col.as<int32_t>();
  if (!c->P_int && !c->P_ext) launch_zero(t2, 2 * vs * nrhs, c->stream);
  // FP32 values when the preconditioner was assembled MIXED: for many
  // right-hand sides the matrix-core product on their block-sparse copy
  // (columns over the union, rows of the block)
  const bool pbsr = many && (c->PSi32.p || c->PSe32.p);
  if (pbsr) launch_zero(t2, 2 * vs * nrhs, c->stream);
  auto spmv = [&](const int64_t* rpp, const DBuf& S64, const DBuf& C64, const DBuf& S32, const DBuf& C32, int rows,
                  double kr, double ki, const double* xD, const double* xN, double* yD, double* yN, bool acc,
                  BsrHold* bh) {
    if (pbsr && S32.p) {
      if (!bh->valid)
        build_bsr(c, rpp, cl, rows, int(E), S32.as<float>(), c->P_C ? C32.as<float>() : nullptr, true, *bh);
      float* B1 = Bw;
      float* B2 = Bw + size_t(4) * nrhs * 2 * size_t(bh->m.nbc) * BSR_T;
      launch_bsr_pmchwt(bh->m, rows, int(E), kr, ki, xD, xN, yD, yN, nrhs, vs, B1, B2, c->stream);
    } else if (S32.p)
      launch_spmv_pmchwt<float>(rpp, cl, S32.as<float>(), c->P_C ? C32.as<float>() : nullptr, rows, kr, ki, xD, xN, yD,
                                yN, nrhs, vs, c->stream, acc);
    else
      launch_spmv_pmchwt<double>(rpp, cl, S64.as<double>(), c->P_C ? C64.as<double>() : nullptr, rows, kr, ki, xD, xN,
                                 yD, yN, nrhs, vs, c->stream, acc);
  };
  if (c->P_int) {
    if (c->bsrPi.size() != c->sc.size()) c->bsrPi.resize(c->sc.size());
    for (size_t m = 0; m < c->sc.size(); ++m) {
      const Scat& s = c->sc[m];
      const int64_t o = s.edge_off;
      spmv(rp + o, c->PSi, c->PCi, c->PSi32, c->PCi32, s.topo.E, s.k.real(), s.k.imag(), t1, t1 + 2 * E, t2 + 2 * o,
           t2 + 2 * (E + o), false, &c->bsrPi[m]);
    }
  }
  if (c->P_ext)
    spmv(rp, c->PSe, c->PCe, c->PSe32, c->PCe32, int(E), c->k_ext, 0.0, t1, t1 + 2 * E, t2, t2 + 2 * E, c->P_int,
         &c->bsrPe);
  for (size_t m = 0; m < c->sc.size(); ++m) mass_inv(m, true, -1.0, t2, z);
  HIPCHK(hipGetLastError());
}

// Device table of the scatterers' first union edges (and E_tot) for the
// layout kernel, rebuilt when the scatterers change.
const int32_t* scat_offsets(pmchwt_ctx* c) {
  if (c->soff_n != int(c->sc.size()) || c->soff_E != c->E_tot) {
    std::vector<int32_t> o;
    for (auto& s : c->sc) o.push_back(s.edge_off);
    o.push_back(int32_t(c->E_tot));
    c->soff = upload(c, o);
    c->soff_n = int(c->sc.size());
    c->soff_E = c->E_tot;
  }
  return c->soff.as<int32_t>();
}

// Stream order between a caller's stream (device-pointer entry points; null:
// none) and the context's: the context's work waits for what the caller has
// enqueued so far, and the caller's later work waits for the context's.
void stream_wait(hipStream_t waiter, hipStream_t on) {
  hipEvent_t e = nullptr;
  HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  HIPCHK(hipEventRecord(e, on));
  HIPCHK(hipStreamWaitEvent(waiter, e, 0));
  HIPCHK(hipEventDestroy(e));
}
void order_before_ctx(pmchwt_ctx* c, void* user) {
  hipStream_t u = static_cast<hipStream_t>(user);
  if (u && u != c->stream) stream_wait(c->stream, u);
}
void order_after_ctx(pmchwt_ctx* c, void* user) {
  hipStream_t u = static_cast<hipStream_t>(user);
  if (u && u != c->stream) stream_wait(u, c->stream);
}

// API layout (scatterer-major [D_m ; N_m]) <-> internal layout ([D ; N] over the union)
void to_internal(const pmchwt_ctx* c, const pmchwt_complex* in, int nrhs, std::vector<double>& out) {
  const int64_t E = c->E_tot, N = 2 * E;
  out.assign(size_t(2 * N * nrhs), 0.0);
  for (int r = 0; r < nrhs; ++r)
    for (auto& s : c->sc)
      for (int e = 0; e < s.topo.E; ++e)
        for (int comp = 0; comp < 2; ++comp) {
          const pmchwt_complex v = in[r * N + 2 * int64_t(s.edge_off) + comp * s.topo.E + e];
          const int64_t k = r * N + comp * E + s.edge_off + e;
          out[2 * k] = v.re;
          out[2 * k + 1] = v.im;
        }
}

void to_api(const pmchwt_ctx* c, const std::vector<double>& in, int nrhs, pmchwt_complex* out) {
  const int64_t E = c->E_tot, N = 2 * E;
  for (int r = 0; r < nrhs; ++r)
    for (auto& s : c->sc)
      for (int e = 0; e < s.topo.E; ++e)
        for (int comp = 0; comp < 2; ++comp) {
          const int64_t k = r * N + comp * E + s.edge_off + e;
          out[r * N + 2 * int64_t(s.edge_off) + comp * s.topo.E + e] = {in[2 * k], in[2 * k + 1]};
        }
}

// Solve G x_q = b_q for nvec complex vectors (length n, stride `stride`
// complex) by conjugate gradients; G real symmetric positive definite, dense.
// x = G^-1 b for the rows [0, n) of one scatterer; rowptr points at its first
// row (absolute offsets into col / val)
void gram_cg(pmchwt_ctx* c, const int64_t* rowptr, int n, const double* b_in, double* x_out, int64_t in_stride,
             int nvec) {
  // one workgroup per vector runs the whole iteration: no host round trip
  DBuf work = dalloc_c<double>(c, 6 * size_t(n) * nvec);
  launch_gram_cg(rowptr, c->g_col.as<int32_t>(), c->g_val.as<double>(), n, b_in, in_stride, x_out, in_stride, nvec,
                 work.as<double>(), 1e-28, 1000, c->stream);
  HIPCHK(hipGetLastError());
}

// Galerkin right-hand side into device buffer b (internal layout)
// Plane-wave data on the device: directions (3 per wave) and polarisations
// (re, im per component)
void upload_waves(pmchwt_ctx* c, const double* dirs, const pmchwt_complex* pols, int nrhs, DBuf& dd, DBuf& dp) {
  std::vector<double> hp(6 * size_t(nrhs));
  for (int r = 0; r < nrhs; ++r)
    for (int d = 0; d < 3; ++d) {
      hp[6 * r + 2 * d] = pols[3 * r + d].re;
      hp[6 * r + 2 * d + 1] = pols[3 * r + d].im;
    }
  std::vector<double> hd(dirs, dirs + 3 * size_t(nrhs));
  dd = upload(c, hd);
  dp = upload(c, hp);
}

// Incident-field projections (device buffers, internal layout): g_i = int
// u^inc . (n x rwg_i) and c_inc = G^-1 int u^inc . rwg_i (the L2 projection
// onto RWG, G the RWG Gram matrix)
void incident_projection(pmchwt_ctx* c, const double* dirs, const pmchwt_complex* pols, int nrhs, double* g_out,
                         double* cinc_out) {
  const int64_t E = c->E_tot, vs = vlen(c);
  DBuf dd, dp;
  upload_waves(c, dirs, pols, nrhs, dd, dp);
  DBuf h = dalloc_c<double>(c, size_t(2 * vs * nrhs));
  launch_zero(g_out, 2 * vs * nrhs, c->stream);
  launch_zero(h.as<double>(), 2 * vs * nrhs, c->stream);
  RhsJob j{};
  j.F = c->F_tot;
  j.nrhs = nrhs;
  j.dirs = dd.as<double>();
  j.pols = dp.as<double>();
  j.k_ext = c->k_ext;
  j.E_tot = E;
  j.g = g_out;
  j.h = h.as<double>();
  launch_rhs(asm_params<double>(c), j, c->stream);
  HIPCHK(hipGetLastError());
  // c_inc = G^-1 h per scatterer: batched conjugate gradients on the SPD
  // RWG Gram matrix (both components of every wave at once)
  for (size_t m = 0; m < c->sc.size(); ++m) {
    const Scat& s = c->sc[m];
    gram_cg(c, c->g_rowptr.as<int64_t>() + s.edge_off, s.topo.E, h.as<double>() + 2 * int64_t(s.edge_off),
            cinc_out + 2 * int64_t(s.edge_off), E, 2 * nrhs);
  }
}

// b = g/2 - A^i c_inc; g_keep / cinc_keep (optional, 2 vs nrhs doubles each)
// receive g and c_inc for a later FP64 residual
void build_rhs(pmchwt_ctx* c, const double* dirs, const pmchwt_complex* pols, int nrhs, double* b,
               bool fp64_interior = false, DBuf* g_keep = nullptr, DBuf* cinc_keep = nullptr) {
  const int64_t E = c->E_tot, vs = vlen(c);
  DBuf g = dalloc_c<double>(c, size_t(2 * vs * nrhs)), cinc = dalloc_c<double>(c, size_t(2 * vs * nrhs)),
       t = dalloc_c<double>(c, size_t(2 * vs * nrhs));
  incident_projection(c, dirs, pols, nrhs, g.as<double>(), cinc.as<double>());
  // b = g/2 - A^i c_inc
  if (fp64_interior) {
    apply_A_free(c, cinc.as<double>(), t.as<double>(), nrhs, false);
  } else {
    launch_zero(t.as<double>(), 2 * vs * nrhs, c->stream);
  }
  if (!fp64_interior) ensure_lower(c, 12);
  for (size_t m = 0; m < c->sc.size() && !fp64_interior; ++m) {
    const Scat& s = c->sc[m];
    const int64_t o = s.edge_off;
    const double* x = cinc.as<double>();
    double* y = t.as<double>();
    if (nrhs >= MFMA_MIN_RHS && c->precA == PMCHWT_FP64) {  // matrix cores for many right-hand sides
      double* B1 = mfma_ws64(c, nrhs);
      launch_mfma64_pmchwt(c->Si[m].as<double>(), c->Ci[m].as<double>(), c->ldI[m], s.topo.E, s.topo.E, s.k.real(),
                           s.k.imag(), x + 2 * o, x + 2 * (E + o), y + 2 * o, y + 2 * (E + o), nrhs, vs, B1,
                           B1 + size_t(4) * nrhs * 2 * size_t(c->ldE), c->stream);
    } else if (nrhs >= MFMA_MIN_RHS) {
      float* B1 = mfma_ws(c, nrhs);
      launch_mfma_pmchwt(c->Si[m].as<float>(), c->Ci[m].as<float>(), c->ldI[m], s.topo.E, s.topo.E, s.k.real(),
                         s.k.imag(), x + 2 * o, x + 2 * (E + o), y + 2 * o, y + 2 * (E + o), nrhs, vs, B1,
                         B1 + size_t(4) * nrhs * 2 * size_t(c->ldE), c->stream);
    } else if (c->precA == PMCHWT_FP64)
      launch_gemv_pmchwt<double>(c->Si[m].as<double>(), c->Ci[m].as<double>(), c->ldI[m], s.topo.E, s.topo.E,
                                 s.k.real(), s.k.imag(), x + 2 * o, x + 2 * (E + o), y + 2 * o, y + 2 * (E + o), nrhs,
                                 vs, c->stream);
    else
      launch_gemv_pmchwt<float>(c->Si[m].as<float>(), c->Ci[m].as<float>(), c->ldI[m], s.topo.E, s.topo.E, s.k.real(),
                                s.k.imag(), x + 2 * o, x + 2 * (E + o), y + 2 * o, y + 2 * (E + o), nrhs, vs,
                                c->stream);
  }
  HIPCHK(hipMemcpyAsync(b, g.p, size_t(2 * vs * nrhs) * 8, hipMemcpyDeviceToDevice, c->stream));
  launch_axpby(b, t.as<double>(), vs, int(vs), nrhs, 0.5, -1.0, c->stream);
  HIPCHK(hipGetLastError());
  if (g_keep) *g_keep = std::move(g);
  if (cinc_keep) *cinc_keep = std::move(cinc);
  HIPCHK(hipStreamSynchronize(c->stream));
}

// ---------------------------------------------------------------------------
// Batched restarted GMRES on  Op = Ptilde A  (Ptilde = I for P = I),
// classical Gram-Schmidt with one re-orthogonalisation pass (CGS2).
// Reading: the paper does not state the orthogonalisation; CGS2 has the
// stability of modified Gram-Schmidt and maps onto two batched products.
// A true residual is recomputed at the end of every full cycle (the
// floor(R/rho) term of Table 1).
// ---------------------------------------------------------------------------
struct GmresOut {
  std::vector<int> iters, restarts;
  std::vector<double> relres;
  std::vector<int> converged;
};

void op_apply(pmchwt_ctx* c, const double* x, double* y, double* s1, double* s2, double* s3, int nrhs) {
  if (c->precond == PMCHWT_P_I) {
    apply_A(c, x, y, nrhs);
    return;
  }
  apply_A(c, x, s1, nrhs);
  apply_Ptilde(c, s1, y, s2, s3, nrhs);
}

// Pinned host buffers for the small per-iteration transfers: copies from and
// to them are asynchronous (several runs can overlap on the device), and with
// hipHostMallocCoherent the device writes them directly through `dev`.
struct PinnedBuf {
  void* p = nullptr;
  void* dev = nullptr;  // the device's address of the same memory
  explicit PinnedBuf(size_t bytes, unsigned flags = hipHostMallocDefault) {
    if (hipHostMalloc(&p, bytes, flags) != hipSuccess || hipHostGetDevicePointer(&dev, p, 0) != hipSuccess) {
      (void)hipGetLastError();
      throw Fail{PMCHWT_ERR_OUT_OF_MEMORY, "pinned host allocation failed"};
    }
  }
  PinnedBuf(const PinnedBuf&) = delete;
  PinnedBuf& operator=(const PinnedBuf&) = delete;
  ~PinnedBuf() {
    if (p) (void)hipHostFree(p);
  }
};

// Tolerance of a refinement correction solve for one right-hand side whose
// preconditioned residual is nr against nb for the right-hand side itself:
// the correction needs to bring the residual to tol nb only (half of it, for
// the FP32 error of the correction), i.e. reduce nr by 0.5 tol nb / nr, and
// at least by tol (the plain criterion); 1 when the residual already meets
// tol (nothing to solve).
double correction_tol(double tol, double nr, double nb) {
  if (!(nr > tol * nb)) return 1.0;
  return std::max(tol, 0.5 * tol * nb / nr);
}

// One restarted GMRES run as a resumable state machine.  Every step needs one
// application of Op (input op_in(), output op_out(), done by the caller), then
// stage1(), stage2(), stage3() in that order.  Between stages the run only
// enqueues work on the context's stream and waits at the start of the next
// stage for what it needs on the host, so several runs advanced stage by
// stage overlap on the device.  The blocking gmres() below drives one run.
//
// Arnoldi step j (CGS2: two projection passes, the norm and the normalised
// new basis vector) runs entirely on the device.  The host's part of step j
// (Hessenberg column, Givens rotations, residual estimate, convergence) is
// taken one step late, while step j+1 is already queued, so the device never
// waits for the host inside a cycle.  A step queued after the one in which
// every right-hand side converged is discarded (its basis vector is never
// used); a cycle's last step (restart length or iteration limit) is taken
// without look-ahead.  Iterates and iteration counts are those of the
// unlagged method.
struct GmresRun {
  enum Phase { ITER, RESID, DONE };
  pmchwt_ctx* c;
  const double* bt;
  double* x;
  int nrhs, rho, max_iter;
  double tol;
  std::vector<double> tolq;  // per right-hand side
  int64_t vs, vecd, vstep;
  int n;
  double *V, *w, *r, *s1, *s2, *s3, *dpar, *dn;
  DBuf dact, dscale, dy, dupd, dpart;
  PinnedBuf hpin;
  // the two result slots, coherent host memory that the step's last kernel
  // writes directly (no copy launch per step)
  PinnedBuf hres;
  // per-step results on the host, two slots (step j uses slot j & 1):
  // first-pass projections, second-pass projections, norm of the new vector
  double* h_res[2];
  double* d_res[2];  // the same slots as the device addresses them
  int32_t* h_act[2];
  double *h_scale, *h_y, *h_beta;
  int32_t* h_upd;
  hipEvent_t ev = nullptr;
  double seqno = 0, slot_seq[2] = {-1, -1};  // step numbers: last issued, expected per slot
  GmresOut out;
  std::vector<double> bnorm, beta;
  std::vector<int32_t> active, dev_active;  // host view; what the device's mask holds
  std::vector<cd> H, cs, sn, g;
  std::vector<int> jend, done_cycle;
  int total = 0, j = 0;
  bool all_done = false;
  bool pend = false;   // step j-1 queued, its host part not yet taken
  bool ended = false;  // the cycle ended in this step's stage2
  Phase phase = DONE;
  Phase step = DONE;  // phase in which the current step started (set by stage1)

  // partial sums of one step on the device: two projection passes of at most
  // 2 (1024 + (rho+1) nrhs) doubles each, the norm's update_blocks(n) nrhs;
  // the finished values [h1 | h2 | norms] go to the host slots (hres)
  size_t part_doubles() const { return 4 * (1024 + size_t(rho + 1) * nrhs) + size_t(update_blocks(n)) * nrhs; }
  // [h1 | h2 | norms | flags]: the finish kernel sets flags[r] to the step's
  // number after the rest of the slot
  static size_t flag_off(int nrhs, int rho) { return 4 * size_t(rho + 1) * nrhs + nrhs; }
  static size_t res_doubles(int nrhs, int rho) { return flag_off(nrhs, rho) + nrhs; }
  static size_t pinned_bytes(int nrhs, int rho) {
    return 8 * (2 * size_t(nrhs) + 2 * size_t(rho + 1) * nrhs) + 4 * 3 * size_t(nrhs) + 64;
  }
  cd& Hm(int q, int i, int jj) { return H[(size_t(q) * (rho + 1) + i) * rho + jj]; }

  // tolq (optional): a tolerance per right-hand side (>= 1: nothing to do)
  GmresRun(pmchwt_ctx* c_, const double* bt_, double* x_, int nrhs_, double tol_, int rho_, int max_iter_,
           const double* tolq_ = nullptr)
      : c(c_), bt(bt_), x(x_), nrhs(nrhs_), rho(rho_), max_iter(max_iter_), tol(tol_),
        tolq(tolq_ ? std::vector<double>(tolq_, tolq_ + nrhs_) : std::vector<double>(size_t(nrhs_), tol_)),
        hpin(pinned_bytes(nrhs_, rho_)), hres(2 * 8 * res_doubles(nrhs_, rho_), hipHostMallocCoherent) {
    vs = vlen(c);
    n = int(vs);
    vecd = 2 * vs;
    vstep = int64_t(nrhs) * vs;
    const size_t need =
        size_t(rho + 1 + 5) * nrhs * vecd + part_doubles() + 16 * size_t(nrhs);
    double* W = need_work(c, need);
    V = W;
    w = V + size_t(rho + 1) * nrhs * vecd;
    r = w + nrhs * vecd;
    s1 = r + nrhs * vecd;
    s2 = s1 + nrhs * vecd;
    s3 = s2 + nrhs * vecd;
    dpar = s3 + nrhs * vecd;                   // step partial sums
    dn = dpar + part_doubles();                // nrhs doubles, norms outside the cycle
    dact = dalloc_c<int32_t>(c, nrhs);
    dupd = dalloc_c<int32_t>(c, nrhs);
    dscale = dalloc_c<double>(c, nrhs);
    dy = dalloc_c<double>(c, 2 * size_t(rho + 1) * nrhs);
    dpart = dalloc_c<double>(c, 2 * (size_t(rho + 2) * nrhs + 1024));
    double* hp = static_cast<double*>(hpin.p);
    h_res[0] = static_cast<double*>(hres.p);
    h_res[1] = h_res[0] + res_doubles(nrhs, rho);
    d_res[0] = static_cast<double*>(hres.dev);
    d_res[1] = d_res[0] + res_doubles(nrhs, rho);
    h_scale = hp;
    h_y = h_scale + nrhs;
    h_beta = h_y + 2 * size_t(rho + 1) * nrhs;
    h_act[0] = reinterpret_cast<int32_t*>(h_beta + nrhs);
    h_act[1] = h_act[0] + nrhs;
    h_upd = h_act[1] + nrhs;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    for (int sl = 0; sl < 2; ++sl)
      for (int q = 0; q < nrhs; ++q) h_res[sl][flag_off(nrhs, rho) + q] = -1.0;
    out.iters.assign(nrhs, 0);
    out.restarts.assign(nrhs, 0);
    out.relres.assign(nrhs, 1.0);
    out.converged.assign(nrhs, 0);
    bnorm.assign(nrhs, 0.0);
    beta.assign(nrhs, 0.0);
    active.assign(nrhs, 0);
    H.assign(size_t(rho + 1) * rho * nrhs, cd(0));
    cs.assign(size_t(rho) * nrhs, cd(0));
    sn.assign(size_t(rho) * nrhs, cd(0));
    g.assign(size_t(rho + 1) * nrhs, cd(0));
  }
  GmresRun(const GmresRun&) = delete;
  GmresRun& operator=(const GmresRun&) = delete;
  ~GmresRun() {
    // the pinned buffers and small device arrays may still feed queued copies
    (void)hipStreamSynchronize(c->stream);
    if (ev) (void)hipEventDestroy(ev);
  }

  void wait() { HIPCHK(hipEventSynchronize(ev)); }
  // Wait for the results of the step in slot sl: spin on its flags in host
  // memory (no event on the stream between steps).  A stream that has gone
  // idle, or failed, without setting them ends the wait with an error.
  void wait_step(int sl) {
    const volatile double* f = h_res[sl] + flag_off(nrhs, rho);
    const double want = slot_seq[sl];
    auto ready = [&]() {
      for (int q = 0; q < nrhs; ++q)
        if (f[q] != want) return false;
      return true;
    };
    for (int64_t spin = 1; !ready(); ++spin) {
      if ((spin & 1023) != 0) continue;
      const hipError_t e = hipStreamQuery(c->stream);
      if (e == hipErrorNotReady) continue;
      HIPCHK(e);
      if (!ready()) throw Fail{PMCHWT_ERR_DEVICE, "Arnoldi step results did not arrive"};
    }
    std::atomic_thread_fence(std::memory_order_acquire);
  }
  void mark() { HIPCHK(hipEventRecord(ev, c->stream)); }

  // x = 0, r = bt, |bt| (synchronous), then the first cycle
  void start() {
    launch_zero(x, vecd * nrhs, c->stream);
    HIPCHK(hipMemcpyAsync(r, bt, size_t(vecd * nrhs) * 8, hipMemcpyDeviceToDevice, c->stream));
    launch_norms(bt, vs, n, nrhs, dn, c->stream);
    HIPCHK(hipMemcpyAsync(h_beta, dn, 8 * nrhs, hipMemcpyDeviceToHost, c->stream));
    mark();
    wait();
    for (int q = 0; q < nrhs; ++q) {
      bnorm[q] = beta[q] = h_beta[q];
      if (bnorm[q] == 0.0) {
        out.converged[q] = 1;
        out.relres[q] = 0.0;
      } else if (tolq[q] >= 1.0) {
        out.converged[q] = 1;
        out.relres[q] = 1.0;
      }
    }
    begin_cycle();
  }

  // called with nothing of this run left in flight that reads h_act or h_scale
  void begin_cycle() {
    bool any = false;
    for (int q = 0; q < nrhs; ++q) {
      active[q] = !out.converged[q];
      any |= bool(active[q]);
    }
    if (!any || total >= max_iter) {
      phase = DONE;
      return;
    }
    for (int q = 0; q < nrhs; ++q) {
      h_act[0][q] = active[q];
      h_scale[q] = active[q] ? 1.0 / beta[q] : 0.0;
    }
    HIPCHK(hipMemcpyAsync(dact.p, h_act[0], 4 * nrhs, hipMemcpyHostToDevice, c->stream));
    dev_active = active;
    HIPCHK(hipMemcpyAsync(dscale.p, h_scale, 8 * nrhs, hipMemcpyHostToDevice, c->stream));
    launch_scale_copy(r, vs, V, vs, n, nrhs, dscale.as<double>(), c->stream);
    std::fill(H.begin(), H.end(), cd(0));
    std::fill(g.begin(), g.end(), cd(0));
    for (int q = 0; q < nrhs; ++q) g[size_t(q) * (rho + 1)] = beta[q];
    jend.assign(nrhs, 0);
    done_cycle.assign(nrhs, 0);
    j = 0;
    pend = false;
    phase = ITER;
  }

  const double* op_in() const { return phase == ITER ? V + size_t(j) * nrhs * vecd : x; }
  double* op_out() const { return phase == ITER ? w : r; }

  void stage1() {
    step = phase;
    ended = false;
    if (step == ITER) {  // CGS2 (two passes), the norm, v_{j+1} = w / |w|
      // the split reductions stay as partial sums: the update kernels, the
      // normalisation and the host each add them in the same order
      // (the second update also leaves the partial sums of the new norm)
      const int S1 = dots_splits(j + 1, nrhs, n), S2 = update_blocks(n);
      const size_t m = 2 * size_t(S1) * (j + 1) * nrhs;
      double* h1 = dpar;
      double* h2 = dpar + m;
      double* hn = dpar + 2 * m;
      const int32_t* act = dact.as<int32_t>();
      dots_part_only(V, vstep, j + 1, w, vs, n, act, nrhs, vs, h1, c->stream);
      launch_update(V, vstep, j + 1, w, vs, n, act, nrhs, vs, h1, j + 1, -1.0, c->stream, S1);
      dots_part_only(V, vstep, j + 1, w, vs, n, act, nrhs, vs, h2, c->stream);
      launch_update(V, vstep, j + 1, w, vs, n, act, nrhs, vs, h2, j + 1, -1.0, c->stream, S1, hn);
      slot_seq[j & 1] = ++seqno;
      launch_finish_step(w, vs, V + size_t(j + 1) * nrhs * vecd, vs, n, nrhs, hn, S2, act, h1, h2, S1, j + 1,
                         d_res[j & 1], d_res[j & 1] + flag_off(nrhs, rho), seqno, c->stream);
    } else if (step == RESID) {  // r = bt - Op x
      launch_axpby(r, bt, vs, n, nrhs, -1.0, 1.0, c->stream);
      launch_norms(r, vs, n, nrhs, dn, c->stream, dpart.as<double>());
      HIPCHK(hipMemcpyAsync(h_beta, dn, 8 * nrhs, hipMemcpyDeviceToHost, c->stream));
      mark();
    }
  }

  void stage2() {
    if (step == ITER) {  // the host part of the previous step
      if (!pend) return;
      pend = false;
      wait_step((j - 1) & 1);
      if (column(j - 1)) {
        end_cycle(j - 1);
        ended = true;
      }
    } else if (step == RESID) {
      wait();
      for (int q = 0; q < nrhs; ++q) {
        beta[q] = h_beta[q];
        if (out.converged[q] || jend[q] == 0) continue;
        out.restarts[q] += 1;
        out.relres[q] = beta[q] / bnorm[q];
        if (beta[q] / bnorm[q] <= tolq[q]) out.converged[q] = 1;
      }
      begin_cycle();
    }
  }

  void stage3() {
    if (step != ITER || ended) return;
    if (j + 1 >= rho || total + 1 >= max_iter) {  // the cycle's last step: no look-ahead
      wait_step(j & 1);
      column(j);
      end_cycle(j);
      return;
    }
    pend = true;
    ++j;
  }

  // Host part of step jj: Hessenberg column, Givens rotations, residual
  // estimate, per-RHS convergence.  True when the cycle ends after it.
  bool column(int jj) {
    const int sl = jj & 1;
    const size_t m = 2 * size_t(jj + 1) * nrhs;
    const double* h1 = h_res[sl];
    const double* h2 = h1 + m;
    const double* hn = h1 + 2 * m;
    ++total;
    all_done = true;
    for (int q = 0; q < nrhs; ++q) {
      if (!active[q]) continue;
      out.iters[q] += 1;
      for (int i = 0; i <= jj; ++i) {
        const size_t o = 2 * (size_t(q) * (jj + 1) + i);
        Hm(q, i, jj) = cd(h1[o] + h2[o], h1[o + 1] + h2[o + 1]);
      }
      Hm(q, jj + 1, jj) = hn[q];
      for (int i = 0; i < jj; ++i) {
        const cd a = Hm(q, i, jj), b = Hm(q, i + 1, jj);
        const cd c_ = cs[size_t(q) * rho + i], s_ = sn[size_t(q) * rho + i];
        Hm(q, i, jj) = c_ * a + s_ * b;
        Hm(q, i + 1, jj) = -std::conj(s_) * a + std::conj(c_) * b;
      }
      const cd a = Hm(q, jj, jj), b = Hm(q, jj + 1, jj);
      const double den = std::sqrt(std::norm(a) + std::norm(b));
      const cd c_ = den > 0 ? std::conj(a) / den : cd(1), s_ = den > 0 ? std::conj(b) / den : cd(0);
      cs[size_t(q) * rho + jj] = c_;
      sn[size_t(q) * rho + jj] = s_;
      Hm(q, jj, jj) = den;
      Hm(q, jj + 1, jj) = 0;
      cd& gj = g[size_t(q) * (rho + 1) + jj];
      g[size_t(q) * (rho + 1) + jj + 1] = -std::conj(s_) * gj;
      gj = c_ * gj;
      const double res = std::abs(g[size_t(q) * (rho + 1) + jj + 1]) / bnorm[q];
      out.relres[q] = res;
      jend[q] = jj + 1;
      // converged inside the cycle (a convergence exactly at the cycle end
      // still goes through the cycle-end residual, as Table 1 counts it)
      if (res <= tolq[q] && jj + 1 < rho) {
        done_cycle[q] = 1;
        active[q] = 0;
      } else {
        all_done = false;
      }
    }
    // the copy (only when the active set changed) reads slot sl when it runs;
    // the slot is next written by the host part of step jj + 2, after the
    // device has passed step jj + 2
    if (active != dev_active) {
      for (int q = 0; q < nrhs; ++q) h_act[sl][q] = active[q];
      HIPCHK(hipMemcpyAsync(dact.p, h_act[sl], 4 * nrhs, hipMemcpyHostToDevice, c->stream));
      dev_active = active;
    }
    return all_done || jj + 1 >= rho || total >= max_iter;
  }

  // x += V y for every right-hand side that iterated in this cycle; then the
  // cycle-end residual, or done.  Steps queued after jj are discarded.
  void end_cycle(int jj) {
    if (j > jj) {  // step j was queued ahead and is dropped: its products are no matvecs of the method
      c->calls_A -= 1;
      if (c->precond != PMCHWT_P_I) c->calls_P -= 1;
      c->prof.lookahead_discarded += 1;
    }
    pend = false;
    int maxj = 0;
    for (int q = 0; q < nrhs; ++q) {
      const int m = jend[q];
      h_upd[q] = m > 0;
      for (int i = 0; i < 2 * (rho + 1); ++i) h_y[2 * size_t(q) * (rho + 1) + i] = 0.0;
      if (m == 0) continue;
      maxj = std::max(maxj, m);
      std::vector<cd> y(m);
      for (int i = m - 1; i >= 0; --i) {
        cd s = g[size_t(q) * (rho + 1) + i];
        for (int k = i + 1; k < m; ++k) s -= Hm(q, i, k) * y[k];
        y[i] = s / Hm(q, i, i);
      }
      for (int i = 0; i < m; ++i) {
        h_y[2 * (size_t(q) * (rho + 1) + i)] = y[i].real();
        h_y[2 * (size_t(q) * (rho + 1) + i) + 1] = y[i].imag();
      }
    }
    if (maxj > 0) {
      HIPCHK(hipMemcpyAsync(dy.p, h_y, 16 * size_t(rho + 1) * nrhs, hipMemcpyHostToDevice, c->stream));
      HIPCHK(hipMemcpyAsync(dupd.p, h_upd, 4 * nrhs, hipMemcpyHostToDevice, c->stream));
      launch_update(V, vstep, maxj, x, vs, n, dupd.as<int32_t>(), nrhs, vs, dy.as<double>(), rho + 1, 1.0, c->stream);
    }
    for (int q = 0; q < nrhs; ++q)
      if (done_cycle[q]) out.converged[q] = 1;
    bool pending = false;
    for (int q = 0; q < nrhs; ++q) pending |= (!out.converged[q] && jend[q] > 0);
    phase = pending ? RESID : DONE;
  }
};

GmresOut gmres(pmchwt_ctx* c, const double* bt, double* x, int nrhs, double tol, int rho, int max_iter,
               const double* tolq = nullptr) {
  GmresRun g(c, bt, x, nrhs, tol, rho, max_iter, tolq);
  g.start();
  while (g.phase != GmresRun::DONE) {
    op_apply(c, g.op_in(), g.op_out(), g.s1, g.s2, g.s3, nrhs);
    g.stage1();
    g.stage2();
    g.stage3();
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  return g.out;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* pmchwt_version(void) { return "pmchwt-mi355x 0.1 (gfx950)"; }

int pmchwt_create(pmchwt_ctx** out, int device, void* hip_stream) {
  if (!out) return PMCHWT_ERR_INVALID_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return PMCHWT_ERR_DEVICE;
  if (device < 0 || device >= ndev) return PMCHWT_ERR_INVALID_ARG;
  auto* c = new (std::nothrow) pmchwt_ctx();
  if (!c) return PMCHWT_ERR_OUT_OF_MEMORY;
  c->device = device;
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return PMCHWT_ERR_DEVICE;
  }
  if (hip_stream) {
    c->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) {
      delete c;
      return PMCHWT_ERR_DEVICE;
    }
    c->own_stream = true;
  }
  if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_main, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_side, hipEventDisableTiming) != hipSuccess) {
    delete c;
    return PMCHWT_ERR_DEVICE;
  }
  if (rocblas_create_handle(&c->blas) != rocblas_status_success) {
    delete c;
    return PMCHWT_ERR_DEVICE;
  }
  if (scratch_setup(device) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return PMCHWT_ERR_DEVICE;
  }
  rocblas_set_stream(c->blas, c->stream);
  double l[14][3], w[14];
  triangle_rules(l, w);
  if (upload_rules(&l[0][0], w, c->stream) != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) {
    delete c;
    return PMCHWT_ERR_DEVICE;
  }
  *out = c;
  return PMCHWT_OK;
}

int pmchwt_add_scatterer(pmchwt_ctx* c, const double* verts, int32_t nv, const int32_t* tris, int32_t nt,
                         pmchwt_complex eps_r, int32_t* id) {
  return guarded(c, [&]() -> int {
    if (!verts || !tris || nv <= 0 || nt <= 0) return fail(c, PMCHWT_ERR_INVALID_ARG, "null or empty mesh");
    Scat s;
    std::string err;
    if (!build_topology(verts, nv, tris, nt, s.topo, err)) return fail(c, PMCHWT_ERR_INVALID_MESH, err);
    s.eps = cd(eps_r.re, eps_r.im);
    s.edge_off = c->E_tot;
    s.tri_off = c->F_tot;
    s.vert_off = c->nv_tot;
    c->E_tot += s.topo.E;
    c->F_tot += s.topo.F;
    c->nv_tot += s.topo.nv;
    c->sc.push_back(std::move(s));
    c->geo_uploaded = false;
    c->have_A = false;
    c->count_key = -1;
    c->chunk_size = 0;
    c->nf.valid = false;
    c->sing.n = -1;
    c->sym.n = -1;
    c->cells_valid = false;
    c->gram_valid = false;
    c->mp.valid = false;
    c->slabs.clear();
    if (id) *id = int32_t(c->sc.size() - 1);
    return PMCHWT_OK;
  });
}

int pmchwt_set_wavenumber(pmchwt_ctx* c, double k) {
  return guarded(c, [&]() -> int {
    if (!(k > 0.0) || !std::isfinite(k)) return fail(c, PMCHWT_ERR_INVALID_ARG, "k_ext must be positive");
    c->k_ext = k;
    c->have_A = false;
    return PMCHWT_OK;
  });
}

int pmchwt_sizes(const pmchwt_ctx* c, int32_t* ns, int64_t* nu) {
  if (!c) return PMCHWT_ERR_INVALID_ARG;
  if (ns) *ns = int32_t(c->sc.size());
  if (nu) *nu = 2 * int64_t(c->E_tot);
  return PMCHWT_OK;
}

int pmchwt_num_edges(const pmchwt_ctx* c, int32_t m, int32_t* E) {
  if (!c || !E || m < 0 || m >= int32_t(c->sc.size())) return PMCHWT_ERR_INVALID_ARG;
  *E = c->sc[m].topo.E;
  return PMCHWT_OK;
}

int pmchwt_assemble(pmchwt_ctx* c, const pmchwt_assembly_opts* A, const pmchwt_assembly_opts* P,
                    pmchwt_precond kind) {
  return guarded(c, [&]() -> int {
    if (c->sc.empty()) return fail(c, PMCHWT_ERR_STATE, "no scatterer added");
    if (!(c->k_ext > 0)) return fail(c, PMCHWT_ERR_STATE, "wavenumber not set");
    check_opts(A, "A");
    check_opts(P, "P");
    if (int(kind) < 0 || int(kind) > 6) return fail(c, PMCHWT_ERR_INVALID_ARG, "unknown preconditioner");
    c->have_A = false;
    flush_times(c);
    c->prof = pmchwt_profile{};
    c->a64.valid = false;
    c->a64.Se = DBuf();
    c->a64.Ce = DBuf();
    c->a64.Si.clear();
    c->a64.Ci.clear();
    const double w0 = wall_ms();
    build_duals(c);
    c->prof.wall_dual = wall_ms() - w0;
    upload_geometry(c);
    upload_k(c);
    c->optA = *A;
    c->optP = *P;
    c->precA = A->precision;
    const double w1 = wall_ms();
    if (A->precision == PMCHWT_FP64)
      assemble_A_impl<double>(c, *A);
    else
      assemble_A_impl<float>(c, *A);
    HIPCHK(hipStreamSynchronize(c->stream));
    const double w2 = wall_ms();
    if (!c->cells_valid) {
      const double wt = wall_ms();
      upload_cells(c, c->cells);
      c->cells_valid = true;
      c->prof.wall_dual += wall_ms() - wt;
    }
    CellDev& cells = c->cells;
    c->mass_f32 = P->precision == PMCHWT_MIXED;
    assemble_P_impl(c, *P, int(kind), cells);
    HIPCHK(hipStreamSynchronize(c->stream));
    const double w3 = wall_ms();
    assemble_mass_impl(c, cells);
    HIPCHK(hipStreamSynchronize(c->stream));
    const double w4 = wall_ms();
    c->prof.wall_setup = w1 - w0;
    c->prof.wall_A = w2 - w1;
    c->prof.wall_P = w3 - w2;
    c->prof.wall_mass = w4 - w3;
    c->have_A = true;
    return PMCHWT_OK;
  });
}

int pmchwt_get_block(pmchwt_ctx* c, pmchwt_opkind op, pmchwt_medium med, pmchwt_space sp, int32_t m, int32_t l,
                     pmchwt_complex* out, int64_t ld) {
  return guarded(c, [&]() -> int {
    if (!c->have_A) return fail(c, PMCHWT_ERR_STATE, "not assembled");
    const int M = int(c->sc.size());
    if (!out || m < 0 || l < 0 || m >= M || l >= M) return fail(c, PMCHWT_ERR_INVALID_ARG, "bad block index");
    if (med == PMCHWT_INT && m != l) return fail(c, PMCHWT_ERR_INVALID_ARG, "interior operators are block diagonal");
    const Scat& sm = c->sc[m];
    const Scat& sl = c->sc[l];
    const int Em = sm.topo.E, El = sl.topo.E;
    if (ld < El) return fail(c, PMCHWT_ERR_INVALID_ARG, "ld too small");
    if (sp == PMCHWT_RWG) {
      ensure_lower(c, 15);
      const DBuf* src;
      int64_t sld, r0, c0;
      if (med == PMCHWT_EXT) {
        src = op == PMCHWT_OP_S ? &c->Se : &c->Ce;
        sld = c->ldE;
        r0 = sm.edge_off;
        c0 = sl.edge_off;
      } else {
        src = op == PMCHWT_OP_S ? &c->Si[m] : &c->Ci[m];
        sld = c->ldI[m];
        r0 = 0;
        c0 = 0;
      }
      const size_t es = c->precA == PMCHWT_FP64 ? 16 : 8;
      std::vector<char> buf(size_t(Em) * El * es);
      HIPCHK(hipMemcpy2DAsync(buf.data(), El * es, static_cast<char*>(src->p) + (r0 * sld + c0) * es, sld * es, El * es,
                              Em, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
      for (int i = 0; i < Em; ++i)
        for (int j = 0; j < El; ++j) {
          if (es == 16) {
            const double* p = reinterpret_cast<const double*>(buf.data()) + 2 * (size_t(i) * El + j);
            out[i * ld + j] = {p[0], p[1]};
          } else {
            const float* p = reinterpret_cast<const float*>(buf.data()) + 2 * (size_t(i) * El + j);
            out[i * ld + j] = {p[0], p[1]};
          }
        }
      return PMCHWT_OK;
    }
    const DBuf* v = nullptr;
    if (med == PMCHWT_INT) v = op == PMCHWT_OP_S ? &c->PSi : &c->PCi;
    else v = op == PMCHWT_OP_S ? &c->PSe : &c->PCe;
    if (!v->p) return fail(c, PMCHWT_ERR_STATE, "this BC operator is not part of the preconditioner");
    host_pattern(c);
    std::vector<double> vals(2 * size_t(c->nnzP));
    HIPCHK(hipMemcpyAsync(vals.data(), v->p, vals.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int i = 0; i < Em; ++i) {
      for (int j = 0; j < El; ++j) out[i * ld + j] = {0, 0};
      const int gi = sm.edge_off + i;
      for (int64_t p = c->h_rowptr[gi]; p < c->h_rowptr[gi + 1]; ++p) {
        const int gj = c->h_col[p];
        if (gj >= sl.edge_off && gj < sl.edge_off + El) out[i * ld + (gj - sl.edge_off)] = {vals[2 * p], vals[2 * p + 1]};
      }
    }
    return PMCHWT_OK;
  });
}

int pmchwt_get_entries(pmchwt_ctx* c, pmchwt_opkind op, pmchwt_medium med, pmchwt_space sp, int32_t m, int32_t l,
                       int64_t n, const int32_t* rows, const int32_t* cols, pmchwt_complex* out) {
  return guarded(c, [&]() -> int {
    if (!c->have_A) return fail(c, PMCHWT_ERR_STATE, "not assembled");
    const int M = int(c->sc.size());
    if (n < 0 || (n > 0 && (!rows || !cols || !out)) || m < 0 || l < 0 || m >= M || l >= M)
      return fail(c, PMCHWT_ERR_INVALID_ARG, "bad arguments");
    if (med == PMCHWT_INT && m != l) return fail(c, PMCHWT_ERR_INVALID_ARG, "interior operators are block diagonal");
    const Scat& sm = c->sc[m];
    const Scat& sl = c->sc[l];
    for (int64_t q = 0; q < n; ++q)
      if (rows[q] < 0 || rows[q] >= sm.topo.E || cols[q] < 0 || cols[q] >= sl.topo.E)
        return fail(c, PMCHWT_ERR_INVALID_ARG, "entry index out of range");
    if (sp == PMCHWT_RWG) {
      ensure_lower(c, 15);
      const size_t es = c->precA == PMCHWT_FP64 ? 16 : 8;
      const DBuf* src = med == PMCHWT_EXT ? (op == PMCHWT_OP_S ? &c->Se : &c->Ce) : (op == PMCHWT_OP_S ? &c->Si[m] : &c->Ci[m]);
      const int64_t sld = med == PMCHWT_EXT ? c->ldE : c->ldI[m];
      const int64_t r0 = med == PMCHWT_EXT ? sm.edge_off : 0, c0 = med == PMCHWT_EXT ? sl.edge_off : 0;
      for (int64_t q = 0; q < n; ++q) {
        char buf[16];
        HIPCHK(hipMemcpyAsync(buf, static_cast<char*>(src->p) + ((r0 + rows[q]) * sld + c0 + cols[q]) * es, es,
                              hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (es == 16) {
          double d[2];
          std::memcpy(d, buf, 16);
          out[q] = {d[0], d[1]};
        } else {
          float f[2];
          std::memcpy(f, buf, 8);
          out[q] = {f[0], f[1]};
        }
      }
      return PMCHWT_OK;
    }
    const DBuf* v = med == PMCHWT_INT ? (op == PMCHWT_OP_S ? &c->PSi : &c->PCi) : (op == PMCHWT_OP_S ? &c->PSe : &c->PCe);
    if (!v->p) return fail(c, PMCHWT_ERR_STATE, "this BC operator is not part of the preconditioner");
    host_pattern(c);
    for (int64_t q = 0; q < n; ++q) {
      const int gi = sm.edge_off + rows[q], gj = sl.edge_off + cols[q];
      auto b = c->h_col.begin() + c->h_rowptr[gi], e = c->h_col.begin() + c->h_rowptr[gi + 1];
      auto it = std::lower_bound(b, e, gj);
      if (it == e || *it != gj) {
        out[q] = {0, 0};
        continue;
      }
      const int64_t p = it - c->h_col.begin();
      double d[2];
      HIPCHK(hipMemcpyAsync(d, v->as<double>() + 2 * p, 16, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
      out[q] = {d[0], d[1]};
    }
    return PMCHWT_OK;
  });
}

int pmchwt_get_mass(pmchwt_ctx* c, int32_t m, double* out) {
  return guarded(c, [&]() -> int {
    if (!c->have_A) return fail(c, PMCHWT_ERR_STATE, "not assembled");
    if (!out || m < 0 || m >= int32_t(c->sc.size())) return fail(c, PMCHWT_ERR_INVALID_ARG, "bad arguments");
    const int n = c->sc[m].topo.E;
    const pmchwt_ctx::SparseInv& M = c->MAcsr[m];
    std::vector<int64_t> rp(size_t(n) + 1);
    std::vector<int32_t> col(size_t(std::max<int64_t>(M.nnz, 1)));
    std::vector<double> val(size_t(std::max<int64_t>(M.nnz, 1)));
    HIPCHK(hipMemcpyAsync(rp.data(), M.rowptr.p, rp.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(col.data(), M.col.p, size_t(M.nnz) * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(val.data(), M.val.p, size_t(M.nnz) * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    std::fill(out, out + size_t(n) * n, 0.0);
    for (int r = 0; r < n; ++r)
      for (int64_t p = rp[r]; p < rp[r + 1]; ++p) out[size_t(r) * n + col[p]] = val[p];
    return PMCHWT_OK;
  });
}

int pmchwt_rhs(pmchwt_ctx* c, const double* dirs, const pmchwt_complex* pols, int32_t nrhs, pmchwt_complex* b_out) {
  return guarded(c, [&]() -> int {
    if (!c->have_A) return fail(c, PMCHWT_ERR_STATE, "not assembled");
    if (nrhs <= 0 || !dirs || !pols || !b_out) return fail(c, PMCHWT_ERR_INVALID_ARG, "bad arguments");
    const int64_t vs = vlen(c);
    DBuf b = dalloc_c<double>(c, size_t(2 * vs * nrhs));
    build_rhs(c, dirs, pols, nrhs, b.as<double>());
    std::vector<double> h(size_t(2 * vs * nrhs));
    HIPCHK(hipMemcpy(h.data(), b.p, h.size() * 8, hipMemcpyDeviceToHost));
    to_api(c, h, nrhs, b_out);
    return PMCHWT_OK;
  });
}

int pmchwt_apply_device(pmchwt_ctx* c, int32_t which, const pmchwt_complex* x_dev, int32_t nrhs,
                        pmchwt_complex* y_dev, void* hip_stream) {
  return guarded(c, [&]() -> int {
    if (!c->have_A) return fail(c, PMCHWT_ERR_STATE, "not assembled");
    if (nrhs <= 0 || !x_dev || !y_dev || which < 0 || which > 3) return fail(c, PMCHWT_ERR_INVALID_ARG, "bad arguments");
    const size_t nd = size_t(2 * vlen(c) * nrhs);
    const int32_t* soff = scat_offsets(c);
    const int E = int(c->E_tot), nsc = int(c->sc.size());
    DBuf dx = dalloc_c<double>(c, nd), dy = dalloc_c<double>(c, nd), s1 = dalloc_c<double>(c, nd),
         s2 = dalloc_c<double>(c, nd), s3 = dalloc_c<double>(c, nd);
    order_before_ctx(c, hip_stream);
    launch_layout(reinterpret_cast<const double*>(x_dev), dx.as<double>(), nrhs, E, soff, nsc, true, c->stream);
    if (which == 0)
      apply_A(c, dx.as<double>(), dy.as<double>(), nrhs);
    else if (which >= 2)
      apply_A_free(c, dx.as<double>(), dy.as<double>(), nrhs, which == 2);
    else
      op_apply(c, dx.as<double>(), dy.as<double>(), s1.as<double>(), s2.as<double>(), s3.as<double>(), nrhs);
    launch_layout(dy.as<double>(), reinterpret_cast<double*>(y_dev), nrhs, E, soff, nsc, false, c->stream);
    HIPCHK(hipGetLastError());
    order_after_ctx(c, hip_stream);  // the buffers above return to the pool in stream order
    return PMCHWT_OK;
  });
}

int pmchwt_apply(pmchwt_ctx* c, int32_t which, const pmchwt_complex* x, int32_t nrhs, pmchwt_complex* y) {
  return guarded(c, [&]() -> int {
    if (!c->have_A) return fail(c, PMCHWT_ERR_STATE, "not assembled");
    if (nrhs <= 0 || !x || !y || which < 0 || which > 3) return fail(c, PMCHWT_ERR_INVALID_ARG, "bad arguments");
    const int64_t vs = vlen(c);
    std::vector<double> h;
    to_internal(c, x, nrhs, h);
    DBuf dx = upload(c, h), dy = dalloc_c<double>(c, h.size()), s1 = dalloc_c<double>(c, h.size()),
         s2 = dalloc_c<double>(c, h.size()), s3 = dalloc_c<double>(c, h.size());
    if (which == 0)
      apply_A(c, dx.as<double>(), dy.as<double>(), nrhs);
    else if (which >= 2)
      apply_A_free(c, dx.as<double>(), dy.as<double>(), nrhs, which == 2);
    else
      op_apply(c, dx.as<double>(), dy.as<double>(), s1.as<double>(), s2.as<double>(), s3.as<double>(), nrhs);
    HIPCHK(hipMemcpyAsync(h.data(), dy.p, h.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    to_api(c, h, nrhs, y);
    (void)vs;
    return PMCHWT_OK;
  });
}

// The solve of pmchwt_solve / pmchwt_solve_device: currents to host memory
// (cur) or, in the API layout, to device memory (cur_dev, on the context's
// stream, then ordered before the caller's stream `user`).
static int solve_common(pmchwt_ctx* c, const double* dirs, const pmchwt_complex* pols, int32_t nrhs,
                 const pmchwt_solver_opts* o, pmchwt_complex* cur, pmchwt_complex* cur_dev, void* user,
                 pmchwt_solve_stats* st) {
  return guarded(c, [&]() -> int {
    if (!c->have_A) return fail(c, PMCHWT_ERR_STATE, "not assembled");
    if (nrhs <= 0 || !dirs || !pols || !(cur || cur_dev) || !o) return fail(c, PMCHWT_ERR_INVALID_ARG, "bad arguments");
    if (!(o->tol > 0) || o->restart < 1 || o->restart > 1024 || o->max_iter < 1 || o->ir_max < 0)
      return fail(c, PMCHWT_ERR_INVALID_ARG, "bad solver options");
    const int64_t vs = vlen(c);
    const size_t nd = size_t(2 * vs * nrhs);
    DBuf b = dalloc_c<double>(c, nd), bt = dalloc_c<double>(c, nd), x = dalloc_c<double>(c, nd),
         s1 = dalloc_c<double>(c, nd), s2 = dalloc_c<double>(c, nd), d = dalloc_c<double>(c, nd),
         r = dalloc_c<double>(c, nd);
    flush_times(c);
    EvTimer tm(c->stream);
    c->prof.ms_matvec_total = 0;
    c->prof.ms_matvec_reduce = 0;
    c->prof.matvec_launches = 0;
    c->prof.matvec_timed = 0;
    c->prof.matvec_bytes = 0;
    c->prof.ms_mfma_total = 0;
    c->prof.mfma_launches = 0;
    c->prof.mfma_flops = 0;
    c->prof.lookahead_discarded = 0;
    c->prof.ms_free_apply = 0;
    c->prof.free_launches = 0;
    // a MIXED operator with refinement solves the FP64 system: GMRES starts
    // from the right-hand side of the stored (FP32) interior operators, and
    // every refinement residual r = g/2 - A^i (c_inc + x) - A^e x is one
    // matrix-free FP64 product, so the FP64 right-hand side enters through it
    const bool fp64_ir = c->precA == PMCHWT_MIXED && o->ir_max > 0;
    DBuf g_inc, c_inc;
    build_rhs(c, dirs, pols, nrhs, b.as<double>(), false, fp64_ir ? &g_inc : nullptr, fp64_ir ? &c_inc : nullptr);
    c->calls_A = 0;  // the right-hand side's own interior products are not solver matvecs
    c->calls_P = 0;
    // bt = Ptilde b
    apply_Ptilde(c, b.as<double>(), bt.as<double>(), s1.as<double>(), s2.as<double>(), nrhs);
    GmresOut g = gmres(c, bt.as<double>(), x.as<double>(), nrhs, o->tol, o->restart, o->max_iter);
    int64_t mv_max = 0;
    int it_max = 0, restarts = 0;
    for (int q = 0; q < nrhs; ++q) {
      const int64_t mv = (A_matvecs(c) + P_matvecs(c)) * (g.iters[q] + g.restarts[q]) + P_matvecs(c);
      mv_max = std::max(mv_max, mv);
      it_max = std::max(it_max, g.iters[q]);
      restarts = std::max(restarts, g.restarts[q]);
    }
    // iterative refinement: r = b - A x in FP64 accumulation, then a
    // correction solve while the preconditioned residual exceeds tol, at most
    // ir_max corrections; with refinement the final convergence flag and
    // residual are those of this FP64 check
    int ir = 0;
    while (o->ir_max > 0) {
      if (fp64_ir) {
        // u = c_inc + x (in d), r = g/2 - (A^i u + A^e x)
        HIPCHK(hipMemcpyAsync(d.p, c_inc.p, nd * 8, hipMemcpyDeviceToDevice, c->stream));
        launch_axpby(d.as<double>(), x.as<double>(), vs, int(vs), nrhs, 1.0, 1.0, c->stream);
        apply_A_resid(c, x.as<double>(), d.as<double>(), r.as<double>(), nrhs);
        launch_axpby(r.as<double>(), g_inc.as<double>(), vs, int(vs), nrhs, -1.0, 0.5, c->stream);
      } else {
        apply_A(c, x.as<double>(), r.as<double>(), nrhs);
        launch_axpby(r.as<double>(), b.as<double>(), vs, int(vs), nrhs, -1.0, 1.0, c->stream);
      }
      apply_Ptilde(c, r.as<double>(), s1.as<double>(), s2.as<double>(), d.as<double>(), nrhs);
      std::vector<double> nr(nrhs), nb(nrhs);
      DBuf dn = dalloc_c<double>(c, 2 * nrhs);
      launch_norms(s1.as<double>(), vs, int(vs), nrhs, dn.as<double>(), c->stream);
      launch_norms(bt.as<double>(), vs, int(vs), nrhs, dn.as<double>() + nrhs, c->stream);
      HIPCHK(hipMemcpyAsync(nr.data(), dn.p, 8 * nrhs, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipMemcpyAsync(nb.data(), dn.as<double>() + nrhs, 8 * nrhs, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
      bool ok = true;
      std::vector<double> tq(nrhs);
      for (int q = 0; q < nrhs; ++q) {
        const bool okq = nr[q] <= o->tol * nb[q];
        ok &= okq;
        g.relres[q] = nb[q] > 0 ? nr[q] / nb[q] : 0.0;
        g.converged[q] = okq ? 1 : 0;
        tq[q] = correction_tol(o->tol, nr[q], nb[q]);
      }
      if (ok || ir == o->ir_max) break;
      HIPCHK(hipMemcpyAsync(r.p, s1.p, nd * 8, hipMemcpyDeviceToDevice, c->stream));
      GmresOut g2 = gmres(c, r.as<double>(), d.as<double>(), nrhs, o->tol, o->restart, o->max_iter, tq.data());
      launch_axpby(x.as<double>(), d.as<double>(), vs, int(vs), nrhs, 1.0, 1.0, c->stream);
      int mi = 0;
      for (int q = 0; q < nrhs; ++q) mi = std::max(mi, g2.iters[q]);
      it_max += mi;
      ++ir;
    }
    const double ms = tm.stop();
    flush_times(c);
    mv_max = c->calls_A * A_matvecs(c) + c->calls_P * P_matvecs(c);
    if (cur_dev) {
      launch_layout(x.as<double>(), reinterpret_cast<double*>(cur_dev), nrhs, int(c->E_tot), scat_offsets(c),
                    int(c->sc.size()), false, c->stream);
      HIPCHK(hipGetLastError());
      order_after_ctx(c, user);
      HIPCHK(hipStreamSynchronize(c->stream));
    } else {
      std::vector<double> h(nd);
      HIPCHK(hipMemcpyAsync(h.data(), x.p, nd * 8, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
      to_api(c, h, nrhs, cur);
    }
    bool conv = true;
    double worst = 0;
    for (int q = 0; q < nrhs; ++q) {
      conv &= bool(g.converged[q]);
      worst = std::max(worst, g.relres[q]);
    }
    if (st) {
      st->iterations = it_max;
      st->converged = conv;
      st->matvecs = mv_max;
      st->rel_residual = worst;
      st->ir_steps = ir;
      st->restarts = restarts;
      st->ms_solve = ms;
    }
    if (!conv) return fail(c, PMCHWT_ERR_NOT_CONVERGED, "GMRES reached max_iter");
    return PMCHWT_OK;
  });
}

int pmchwt_solve(pmchwt_ctx* c, const double* dirs, const pmchwt_complex* pols, int32_t nrhs,
                 const pmchwt_solver_opts* o, pmchwt_complex* cur, pmchwt_solve_stats* st) {
  return solve_common(c, dirs, pols, nrhs, o, cur, nullptr, nullptr, st);
}

int pmchwt_solve_device(pmchwt_ctx* c, const double* dirs, const pmchwt_complex* pols, int32_t nrhs,
                        const pmchwt_solver_opts* o, pmchwt_complex* currents_dev, pmchwt_solve_stats* st,
                        void* hip_stream) {
  if (!currents_dev) return fail(c, PMCHWT_ERR_INVALID_ARG, "bad arguments");
  return solve_common(c, dirs, pols, nrhs, o, nullptr, currents_dev, hip_stream, st);
}

// Host currents (API layout: nrhs vectors of 2 E_tot complex, scatterer-major)
// copied as they are and put into the internal layout on the device.
DBuf upload_currents(pmchwt_ctx* c, const pmchwt_complex* cur, int nrhs) {
  const size_t n_api = size_t(nrhs) * 2 * size_t(c->E_tot);
  DBuf dapi = dalloc_c<double>(c, 2 * n_api);
  HIPCHK(hipMemcpyAsync(dapi.p, cur, n_api * sizeof(pmchwt_complex), hipMemcpyHostToDevice, c->stream));
  DBuf dx = dalloc_c<double>(c, size_t(2 * vlen(c) * nrhs));
  launch_layout(dapi.as<double>(), dx.as<double>(), nrhs, int(c->E_tot), scat_offsets(c), int(c->sc.size()), true,
                c->stream);
  return dx;
}

// Far field of nrhs current vectors (device, internal layout) at nobs
// directions into F_out (6 doubles per direction and rhs): the FP64 matrix
// cores for many right-hand sides, else the VALU sum.
constexpr int FAR_MFMA_MIN_RHS = 8;
void far_field_dev(pmchwt_ctx* c, const double* x, int nrhs, const double* obs, int nobs, double* F_out) {
  const AsmParams<double> g = asm_params<double>(c);
  if (nrhs >= FAR_MFMA_MIN_RHS) {
    const FarMfmaPlan fp = far_mfma_plan(c->F_tot, nrhs, nobs);
    DBuf wy = dalloc_c<double>(c, 4 * size_t(fp.npts)), wj = dalloc_c<double>(c, 12 * size_t(fp.npts) * nrhs),
         wb = dalloc_c<double>(c, size_t(fp.n_B)), wp = dalloc_c<double>(c, size_t(fp.n_part));
    launch_far_field_mfma(g, x, c->E_tot, nrhs, c->k_ext, obs, nobs, F_out, fp, wy.as<double>(), wj.as<double>(),
                          wb.as<double>(), wp.as<double>(), c->stream);
  } else {
    const FarPlan fp = far_field_plan(c->F_tot, nrhs, nobs);
    DBuf wy = dalloc_c<double>(c, fp.n_ypts), wj = dalloc_c<double>(c, fp.n_J), wp = dalloc_c<double>(c, fp.n_part);
    launch_far_field(g, x, c->E_tot, nrhs, c->k_ext, obs, nobs, F_out, fp, wy.as<double>(), wj.as<double>(),
                     wp.as<double>(), c->stream);
  }
  HIPCHK(hipGetLastError());
}

// Far field of nrhs >= FAR_MFMA_MIN_RHS current vectors at nh directions and
// their antipodes (F_out: 2 nh directions per rhs, the antipodes second).
void far_field_pair_dev(pmchwt_ctx* c, const double* x, int nrhs, const double* obs, int nh, double* F_out) {
  const FarMfmaPlan fp = far_pair_plan(c->F_tot, nrhs, nh);
  DBuf wy = dalloc_c<double>(c, 4 * size_t(fp.npts)), wj = dalloc_c<double>(c, 12 * size_t(fp.npts) * nrhs),
       wb = dalloc_c<double>(c, size_t(fp.n_B)), wp = dalloc_c<double>(c, size_t(fp.n_part));
  launch_far_field_pair(asm_params<double>(c), x, c->E_tot, nrhs, c->k_ext, obs, nh, F_out, fp, wy.as<double>(),
                        wj.as<double>(), wb.as<double>(), wp.as<double>(), c->stream);
  HIPCHK(hipGetLastError());
}

int pmchwt_far_field_device(pmchwt_ctx* c, const pmchwt_complex* currents_dev, int32_t nrhs, const double* obs_dev,
                            int32_t nobs, pmchwt_complex* F_dev, void* hip_stream) {
  return guarded(c, [&]() -> int {
    if (c->sc.empty() || !(c->k_ext > 0)) return fail(c, PMCHWT_ERR_STATE, "no problem defined");
    if (nrhs <= 0 || nobs <= 0 || !currents_dev || !obs_dev || !F_dev)
      return fail(c, PMCHWT_ERR_INVALID_ARG, "bad arguments");
    upload_geometry(c);
    const int32_t* soff = scat_offsets(c);
    DBuf dx = dalloc_c<double>(c, size_t(2 * vlen(c) * nrhs));
    order_before_ctx(c, hip_stream);
    launch_layout(reinterpret_cast<const double*>(currents_dev), dx.as<double>(), nrhs, int(c->E_tot), soff,
                  int(c->sc.size()), true, c->stream);
    far_field_dev(c, dx.as<double>(), nrhs, obs_dev, nobs, reinterpret_cast<double*>(F_dev));
    order_after_ctx(c, hip_stream);
    return PMCHWT_OK;
  });
}

int pmchwt_far_field(pmchwt_ctx* c, const pmchwt_complex* cur, int32_t nrhs, const double* obs, int32_t nobs,
                     pmchwt_complex* F) {
  return guarded(c, [&]() -> int {
    if (c->sc.empty() || !(c->k_ext > 0)) return fail(c, PMCHWT_ERR_STATE, "no problem defined");
    if (nrhs <= 0 || nobs <= 0 || !cur || !obs || !F) return fail(c, PMCHWT_ERR_INVALID_ARG, "bad arguments");
    upload_geometry(c);
    DBuf dx = upload_currents(c, cur, nrhs);
    std::vector<double> ho(obs, obs + 3 * size_t(nobs));
    DBuf dobs = upload(c, ho), dF = dalloc_c<double>(c, 6 * size_t(nobs) * nrhs);
    far_field_dev(c, dx.as<double>(), nrhs, dobs.as<double>(), nobs, dF.as<double>());
    std::vector<double> hf(6 * size_t(nobs) * nrhs);
    HIPCHK(hipMemcpyAsync(hf.data(), dF.p, hf.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (size_t k = 0; k < hf.size() / 2; ++k) F[k] = {hf[2 * k], hf[2 * k + 1]};
    return PMCHWT_OK;
  });
}

int pmchwt_near_field(pmchwt_ctx* c, const pmchwt_complex* cur, int32_t nrhs, const double* dirs,
                      const pmchwt_complex* pols, const double* pts, int32_t npts, pmchwt_complex* E_out,
                      int32_t* region_out) {
  return guarded(c, [&]() -> int {
    if (!c->have_A) return fail(c, PMCHWT_ERR_STATE, "not assembled");
    if (nrhs <= 0 || npts <= 0 || !cur || !dirs || !pols || !pts || !E_out)
      return fail(c, PMCHWT_ERR_INVALID_ARG, "bad arguments");
    const int64_t vs = vlen(c), nd = 2 * vs * nrhs;
    std::vector<double> h;
    to_internal(c, cur, nrhs, h);
    DBuf dx = upload(c, h), g = dalloc_c<double>(c, size_t(nd)), cinc = dalloc_c<double>(c, size_t(nd));
    incident_projection(c, dirs, pols, nrhs, g.as<double>(), cinc.as<double>());
    DBuf dd, dp;
    upload_waves(c, dirs, pols, nrhs, dd, dp);
    std::vector<int32_t> toff;
    for (auto& s : c->sc) toff.push_back(s.tri_off);
    toff.push_back(c->F_tot);
    std::vector<double> hp(pts, pts + 3 * size_t(npts));
    DBuf dtoff = upload(c, toff), dpts = upload(c, hp), dreg = dalloc_c<int32_t>(c, size_t(npts));
    const int64_t nq = int64_t(c->F_tot) * 6;
    DBuf yp = dalloc_c<double>(c, size_t(4 * nq)), J = dalloc_c<double>(c, size_t(near_j_doubles() * nq * nrhs)),
         dE = dalloc_c<double>(c, 6 * size_t(npts) * nrhs);
    launch_near_field(asm_params<double>(c), dtoff.as<int32_t>(), int(c->sc.size()), dx.as<double>(),
                      cinc.as<double>(), c->E_tot, nrhs, dpts.as<double>(), npts, dd.as<double>(), dp.as<double>(),
                      c->k_ext, c->k_int.as<double>(), dreg.as<int32_t>(), yp.as<double>(), J.as<double>(),
                      dE.as<double>(), c->stream);
    HIPCHK(hipGetLastError());
    std::vector<double> hE(6 * size_t(npts) * nrhs);
    HIPCHK(hipMemcpyAsync(hE.data(), dE.p, hE.size() * 8, hipMemcpyDeviceToHost, c->stream));
    if (region_out)
      HIPCHK(hipMemcpyAsync(region_out, dreg.p, 4 * size_t(npts), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (size_t k = 0; k < hE.size() / 2; ++k) E_out[k] = {hE[2 * k], hE[2 * k + 1]};
    return PMCHWT_OK;
  });
}

int pmchwt_far_field_noalloc(pmchwt_ctx* c, const pmchwt_complex* cur, int32_t nrhs, const double* obs,
                             int32_t nobs, pmchwt_complex* F) {
  return guarded(c, [&]() -> int {
    if (c->sc.empty() || !(c->k_ext > 0)) return fail(c, PMCHWT_ERR_STATE, "no problem defined");
    if (!c->geo_uploaded)
      return fail(c, PMCHWT_ERR_STATE, "geometry not on the device yet (call pmchwt_assemble first)");
    if (nrhs <= 0 || nobs <= 0 || !cur || !obs || !F) return fail(c, PMCHWT_ERR_INVALID_ARG, "bad arguments");
    unsigned char* base = static_cast<unsigned char*>(scratch_address(c->device));
    if (!base) return fail(c, PMCHWT_ERR_DEVICE, "device scratch address not set up");
    // regions of the scratch, each on a 256-byte boundary: currents, directions,
    // F, quadrature points, weighted currents, partial sums
    auto round = [](int64_t doubles) { return (doubles * 8 + 255) / 256 * 256; };
    const int64_t n_x = 4 * int64_t(c->E_tot) * nrhs, n_obs = 3 * int64_t(nobs), n_F = 6 * int64_t(nobs) * nrhs;
    const int64_t npts = int64_t(c->F_tot) * 6;
    const int64_t fixed = round(n_x) + round(n_obs) + round(n_F) + round(4 * npts) + round(12 * npts * nrhs);
    const int64_t cap = int64_t(NOALLOC_SCRATCH_BYTES);
    if (fixed + 256 > cap)
      return fail(c, PMCHWT_ERR_INVALID_ARG,
                  "far field needs more than the " + std::to_string(NOALLOC_SCRATCH_BYTES >> 20) +
                      " MiB device scratch of pmchwt_far_field_noalloc (fewer right-hand sides or directions)");
    const FarPlan fp = far_field_plan_capped(c->F_tot, nrhs, nobs, (cap - fixed) / 8);
    if (fixed + round(fp.n_part) > cap)
      return fail(c, PMCHWT_ERR_INVALID_ARG,
                  "far field needs more than the " + std::to_string(NOALLOC_SCRATCH_BYTES >> 20) +
                      " MiB device scratch of pmchwt_far_field_noalloc (fewer right-hand sides or directions)");
    unsigned char* q = base;
    auto carve = [&](int64_t doubles) {
      double* r = reinterpret_cast<double*>(q);
      q += round(doubles);
      return r;
    };
    double* dx = carve(n_x);
    double* dobs = carve(n_obs);
    double* dF = carve(n_F);
    double* wy = carve(fp.n_ypts);
    double* wj = carve(fp.n_J);
    double* wp = carve(fp.n_part);
    std::vector<double> h;
    to_internal(c, cur, nrhs, h);
    HIPCHK(hipMemcpyAsync(dx, h.data(), h.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(dobs, obs, size_t(n_obs) * 8, hipMemcpyHostToDevice, c->stream));
    // every value the kernels read is written earlier in the same call: no clearing
    launch_far_field(asm_params<double>(c), dx, c->E_tot, nrhs, c->k_ext, dobs, nobs, dF, fp, wy, wj, wp, c->stream);
    HIPCHK(hipGetLastError());
    std::vector<double> hf(static_cast<size_t>(n_F));
    HIPCHK(hipMemcpyAsync(hf.data(), dF, hf.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (size_t k = 0; k < hf.size() / 2; ++k) F[k] = {hf[2 * k], hf[2 * k + 1]};
    return PMCHWT_OK;
  });
}

int pmchwt_cross_sections(pmchwt_ctx* c, const pmchwt_complex* cur, int32_t nrhs, const double* dirs,
                          const pmchwt_complex* pols, double* sext, double* ssca) {
  return guarded(c, [&]() -> int {
    if (c->sc.empty() || !(c->k_ext > 0)) return fail(c, PMCHWT_ERR_STATE, "no problem defined");
    if (nrhs <= 0 || !cur || !dirs || !pols || !sext || !ssca) return fail(c, PMCHWT_ERR_INVALID_ARG, "bad arguments");
    upload_geometry(c);
    // sigma_sca: Gauss-Legendre in cos(theta) x uniform in phi.  The grid is
    // closed under xh -> -xh (symmetric nodes and weights, an even number of
    // phi nodes), so with the matrix cores the far field is formed for the
    // upper half (the nodes of the second half of [0, 1]) and the antipodes.
    const int nth = 64, nph = 128, nobs = nth * nph;
    const bool pairs = nrhs >= FAR_MFMA_MIN_RHS;
    std::vector<double> ct, wt;
    gauss_legendre01(nth, ct, wt);
    std::vector<double> obs(3 * size_t(nobs)), w(nobs);
    const int a0 = pairs ? nth / 2 : 0, nh = (nth - a0) * nph;
    for (int a = a0; a < nth; ++a)
      for (int b = 0; b < nph; ++b) {
        const double cz = 2.0 * ct[a] - 1.0, sz = std::sqrt(std::max(0.0, 1.0 - cz * cz));
        const double ph = 2.0 * M_PI * b / nph;
        const int o = (a - a0) * nph + b;
        obs[3 * o] = sz * std::cos(ph);
        obs[3 * o + 1] = sz * std::sin(ph);
        obs[3 * o + 2] = cz;
        w[o] = 2.0 * wt[a] * (2.0 * M_PI / nph);
        if (pairs) w[nh + o] = w[o];
      }
    obs.resize(3 * size_t(nh));
    DBuf dx = upload_currents(c, cur, nrhs);
    DBuf dobs = upload(c, obs), dw = upload(c, w), dF = dalloc_c<double>(c, 6 * size_t(nobs) * nrhs),
         dsig = dalloc_c<double>(c, nrhs);
    if (pairs)
      far_field_pair_dev(c, dx.as<double>(), nrhs, dobs.as<double>(), nh, dF.as<double>());
    else
      far_field_dev(c, dx.as<double>(), nrhs, dobs.as<double>(), nobs, dF.as<double>());
    launch_sigma_sca(dF.as<double>(), nobs, nrhs, dw.as<double>(), dsig.as<double>(), c->stream);
    std::vector<double> hd(dirs, dirs + 3 * size_t(nrhs));
    DBuf dd = upload(c, hd), dFd = dalloc_c<double>(c, 6 * size_t(nrhs) * nrhs);
    far_field_dev(c, dx.as<double>(), nrhs, dd.as<double>(), nrhs, dFd.as<double>());
    HIPCHK(hipGetLastError());
    std::vector<double> fd(6 * size_t(nrhs) * nrhs);
    HIPCHK(hipMemcpyAsync(ssca, dsig.p, 8 * size_t(nrhs), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(fd.data(), dFd.p, fd.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int r = 0; r < nrhs; ++r) {
      // (4 pi / k) Im(conj(p) . F(d))
      double im = 0.0;
      for (int d = 0; d < 3; ++d) {
        const double fr = fd[6 * (size_t(r) * nrhs + r) + 2 * d], fi = fd[6 * (size_t(r) * nrhs + r) + 2 * d + 1];
        const double pr = pols[3 * r + d].re, pi = pols[3 * r + d].im;
        im += pr * fi - pi * fr;
      }
      sext[r] = 4.0 * M_PI / c->k_ext * im;
    }
    return PMCHWT_OK;
  });
}

int pmchwt_bc_fields(const double* verts, int32_t nv, const int32_t* tris, int32_t nt, int64_t* count, int32_t* ids,
                     double* vals) {
  if (!verts || !tris || !count || nv <= 0 || nt <= 0) return PMCHWT_ERR_INVALID_ARG;
  Topo T;
  DualCells D;
  std::string err;
  if (!build_topology(verts, nv, tris, nt, T, err)) return PMCHWT_ERR_INVALID_MESH;
  if (!build_dual(T, D, err)) return PMCHWT_ERR_INVALID_MESH;
  int64_t n = 0;
  for (int v = 0; v < T.nv; ++v) n += int64_t(D.inc_ptr[v + 1] - D.inc_ptr[v]) * (D.cell_ptr[v + 1] - D.cell_ptr[v]);
  if (!ids || !vals) {
    *count = n;
    return PMCHWT_OK;
  }
  if (*count < n) return PMCHWT_ERR_INVALID_ARG;
  int64_t q = 0;
  for (int v = 0; v < T.nv; ++v) {
    const int n2 = D.cell_ptr[v + 1] - D.cell_ptr[v];
    for (int s = 0; s < n2 / 2; ++s)
      for (int u = 0; u < n2; ++u) {
        const size_t rec = size_t(D.coef_ptr[v]) + size_t(s) * n2 + u;
        ids[2 * q] = D.inc_edges[D.inc_ptr[v] + s];
        ids[2 * q + 1] = D.ring[D.cell_ptr[v] + u];
        for (int k = 0; k < 4; ++k) vals[4 * q + k] = D.coef[4 * rec + k];
        ++q;
      }
  }
  *count = q;
  return PMCHWT_OK;
}

int pmchwt_get_profile(const pmchwt_ctx* c, pmchwt_profile* out) {
  if (!c || !out) return PMCHWT_ERR_INVALID_ARG;
  pmchwt_ctx* m = const_cast<pmchwt_ctx*>(c);  // pending event timings are part of the profile
  return guarded(m, [&]() -> int {
    flush_times(m);
    *out = c->prof;
    return PMCHWT_OK;
  });
}

const char* pmchwt_last_error(const pmchwt_ctx* c) { return c ? c->err.c_str() : "null context"; }

void pmchwt_destroy(pmchwt_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  delete c;
}

}  // extern "C"

#include "serve.inl"
