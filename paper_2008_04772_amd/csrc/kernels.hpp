// Kernel parameter blocks and host launch wrappers of the PMCHWT library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pmchwt {

// Primal triangles of all scatterers (union numbering), SoA.
template <typename M>
struct AsmParams {
  int F;                       // triangles
  const double* tv;            // 9*F: vertex k, component d at (3k+d)*F + t
  const double* tcen;          // 3*F centroids ((P0+P1)+P2)/3
  const double* tdiam2;        // F: max squared edge length
  const double* tarea;         // F
  const int32_t* tvid;         // 3*F vertex ids (global)
  const int32_t* t2e;          // 3*F union edge index of local basis a
  const int8_t* tsgn;          // 3*F sign of local basis a
  const int32_t* tscat;        // F scatterer id
  const int32_t* edge_off;     // per scatterer: first union edge
  const double* k_int;         // per scatterer: interior wavenumber (re, im)
  double k_ext;
  int q_near, q_medium, q_far; // rule orders 1..4
  M* Se;                       // exterior operators, E_tot x E_tot
  M* Ce;
  int64_t ld_ext;
  M** Si;                      // per scatterer interior operators, E_m x E_m
  M** Ci;
  const int64_t* ld_int;
};

// Atomic-free regular-pair assembly.  Trial edges are cut into chunks of
// consecutive edges; for each chunk the distinct trial triangles (T+ and T-
// of its edges) are listed once.  Pass 1 (one workgroup per test triangle and
// chunk) integrates the listed triangles against the test triangle, keeps the
// moments in LDS and writes, for each trial edge j and each local basis a of
// the test triangle, the sum over T+(j), T-(j): a half-reduced row in
// "slot" space (3 slots per test triangle).  Pass 2 adds the two slot rows of
// every test edge into the dense operator.
template <typename M>
struct HalfJob {
  const int32_t* chunk_e;      // nchunks+1: first trial edge of each chunk
  const int32_t* chunk_ptr;    // nchunks+1, into chunk_tri
  const int32_t* chunk_tri;    // distinct trial triangles of each chunk
  const int16_t* edge_map;     // 4 per edge: list position of T+, basis b+, position of T-, basis b-
  const int32_t* edge_scat;    // scatterer of each union edge
  int E_tot;
  int slab_t0;                 // first test triangle of the slab
  M* He_S;                     // slab slot rows x E_tot (exterior S, C)
  M* He_C;
  M* Hi_S;                     // slab slot rows x E_m of the slab's scatterer (interior S, C)
  M* Hi_C;
  int64_t ld_i;                // E_m
  int edge_off_i;              // first union edge of the slab's scatterer
  // upper tiles only (one scatterer stored as symmetric tiles): a workgroup
  // whose chunk lies entirely in tiles left of every edge of its test
  // triangle writes nothing (those entries are the mirror of upper ones)
  int skip_lower;
  const int32_t* t1_tmin;      // per triangle: smallest tile index of its edges
  const int32_t* ch_tmax;      // per chunk: tile index of its last edge
};

// Sauter-Schwab tables per relation kind (1 vertex, 2 edge, 3 identical):
// records (x1, x2, y1, y2, w) on That x That.
struct SingParams {
  int64_t npairs;
  const int32_t* pairs;        // 2*npairs (t1, t2), ordered
  const double* tab[4];
  int npts[4];
  double* blk;                 // FP64 local blocks: per pair, 9 (3a+b) x 4 (Se, Ce, Si, Ci) complex
  // every matrix entry (e_row, e_col) the pairs touch (union indices) and its
  // local-block entries e_item[e_iptr[k] .. e_iptr[k+1]) (9 pair + 3a + b,
  // shifted left by one), in (pair, 3a+b) order
  const int32_t* e_row;
  const int32_t* e_col;
  const int64_t* e_iptr;
  const int32_t* e_item;
  int64_t e_nnz;
};

// Matrix-free FP64 product y = A x (use_ext = 1) or y = A^i x (use_ext = 0)
// over all scatterers; vectors [rhs][D (E_tot); N (E_tot)] complex, vs
// complex entries apart.  Regular pairs are integrated again with the rule
// orders of AsmParams; singular pairs read sing_blk.
struct FreeJob {
  int use_ext;
  int nrhs;
  int E_tot;
  int64_t vs;
  const double* x;             // input of the exterior operators (and of the interior ones if xi is null)
  const double* xi;            // input of the interior operators, or null
  const int64_t* sing_ptr;     // F+1: singular pairs of test triangle t at [sing_ptr[t], sing_ptr[t+1])
  const int32_t* sing_pairs;   // 2 per pair (t1, t2), sorted by t1
  const double* sing_blk;      // SingParams::blk of the same pairs
  double* slots;               // [rhs][3F][yD re, yD im, yN re, yN im]
  const int32_t* edge_slots;   // 2 per union edge: slot 3t+a of T+ and of T-
  double* y;
};
// part: free_part_doubles(F, nrhs) doubles of partial sums (regular pairs by tile)
int64_t free_part_doubles(int F, int nrhs);
void launch_free_apply(const AsmParams<double>& p, const FreeJob& f, double* part, hipStream_t st);

// Sparse approximate inverse of a mass matrix M (one scatterer, n x n): row i
// on the ball of columns within `hops` steps of M's sparsity graph, by a
// Chebyshev iteration for a spectrum in [a, b].  Pass 1 (launch_spinv_ball)
// writes the sorted ball of every row (spinv_cap() columns per row at most)
// and its size (-1 past the capacity); pass 2 (launch_spinv_vals) the CSR
// values at the row pointers orp.  Columns of M may hold spinv_wmax() entries
// at most.
struct SpInvJob {
  int n;
  const int64_t* rp;   // CSR of M (row pointers, columns): the search graph
  const int32_t* ci;
  const int64_t* cp;   // CSC of M (column pointers, rows, values): the gather of (X M)
  const int32_t* ri;
  const double* cv;
  int hops, steps;
  double a, b;
  int32_t* count;      // pass 1: ball sizes
  int32_t* ball;       // pass 1: n x spinv_cap() sorted columns
  const int64_t* orp;  // pass 2: output row pointers, columns, values (float or double), residuals
  int32_t* ocol;
  void* oval;
  double* res;
};
// transpose of an n x n CSR matrix (FP32 values): column counts (cnt zeroed),
// records placed per column (cur zeroed; rec: nnz int64), then, after the
// records are sorted per column (launch_sym_sort), columns and values
void launch_csr_colcount(const int32_t* col, int64_t nnz, int32_t* cnt, hipStream_t st);
void launch_csr_tplace(const int64_t* rowptr, const int32_t* col, int n, const int64_t* trowptr, int32_t* cur,
                       int64_t* rec, hipStream_t st);
void launch_csr_tgather(const int64_t* rec, int64_t nnz, const float* val, int32_t* tcol, float* tval,
                        hipStream_t st);
int spinv_cap();
int spinv_wmax();
void launch_spinv_ball(const SpInvJob& J, int grid, hipStream_t st);
template <typename T>
void launch_spinv_vals(const SpInvJob& J, int grid, hipStream_t st);
void launch_csr_scatter_f32(const int64_t* rowptr, const int32_t* col, const float* val, int n, float* out, int64_t ld,
                            hipStream_t st);

// Dual cells (barycentric rings) of all scatterers.
struct CellParams {
  const int32_t* cell_ptr;     // ncell+1 into ring
  const int32_t* ring;         // global child ids
  const double* child_v;       // 9 per child (AoS)
  const int32_t* child_vid;    // 3 per child, barycentric vertex ids (globally offset)
  const double* child_cen;     // 3 per child
  const double* child_diam2;   // 1 per child
  const double* child_area;    // 1 per child
  const int64_t* coef_ptr;     // ncell+1 (in 4-double records)
  const double* coef;          // (alpha, wx, wy, wz) per (cell, slot, ring position)
  const int32_t* cell_scat;    // scatterer of each cell
};

// Near-field BC operator job: one wavefront per cell pair.
struct BCJob {
  int64_t npairs;
  const int32_t* cpairs;       // 2*npairs (cell v, cell w)
  const int64_t* slot_off;     // npairs+1: offsets into slot_pos
  const int64_t* slot_pos;     // N_v x N_w CSR positions, -1 = dropped by the near-field cutoff
  int want_int, want_ext, want_C;
  int fp32;                    // pair moments and contractions in FP32 (mixed-precision P)
  const double* k_int;         // per scatterer (re, im)
  double k_ext;
  int q_near, q_medium, q_far, n_sing;
  const double* tab[4];
  int npts[4];
  double* out_Si;              // CSR values (re, im) interleaved, FP64
  double* out_Ci;
  double* out_Se;
  double* out_Ce;
  // per slot of every cell pair: the values of the kept entries (nv doubles:
  // re, im of each operator the preconditioner needs, in the order Si, Ci,
  // Se, Ce), which a gather adds per entry over its four slots in a fixed order
  double* slot_val;
  int nv;
  const int64_t* entry_slots;
  int64_t nnz, nslots;
};

// Mass / Gram / right-hand-side / far-field parameter blocks.
struct MassJob {
  int nchild;
  int E;                       // union edges (rows of M_A and M_A^T)
  int64_t nnz_m, nnz_t;
  const int32_t* edge_slots;   // 2 per union edge: 3 T+ + a, 3 T- + a
  const int32_t* child_cell;   // cell of each child
  const int32_t* child_pos;    // ring position
  const int32_t* child_parent; // global primal triangle
  const int32_t* inc_ptr;      // per cell: offset into inc_edges
  const int32_t* inc_edges;    // union edge ids
  const int32_t* edge_scat;    // scatterer of each union edge
  const int32_t* edge_off;     // per scatterer
  // M_A (rows: RWG union edge, columns: scatterer-local BC edge) and M_A^T
  // (rows: BC union edge, columns: scatterer-local RWG edge) as CSR with
  // ascending columns, structural patterns from the mesh adjacency
  const int64_t* m_rowptr;
  const int32_t* m_col;
  double* m_val;
  const int64_t* t_rowptr;
  const int32_t* t_col;
  double* t_val;
  const int64_t* gram_pos;     // RWG Gram: CSR position of local pair (a, b) of triangle t at 9 t + 3 a + b
  double* gram_val;            // RWG Gram CSR values
};

// Structural patterns of M_A and M_A^T (count pass, scan, fill pass).
// Row i of M_A: the BC functions of every edge at a vertex of T+(i) or
// T-(i); row j of M_A^T: the RWG functions of every triangle at an end point
// of edge j.  Columns scatterer-local, ascending.
struct MassPatternJob {
  int E, F;
  int trans;                   // 0: M_A, 1: M_A^T
  const int32_t* edge_slots;   // 2 per union edge: 3 T+ + a, 3 T- + a
  const int32_t* tvid;         // 3*F SoA global vertex ids
  const int32_t* t2e;          // 3*F SoA union edge ids
  const int32_t* inc_ptr;      // per global vertex (cell): edges at it
  const int32_t* inc_edges;
  const int32_t* v2t_ptr;      // per global vertex: triangles at it
  const int32_t* v2t;
  const int32_t* ends;         // 2 per union edge: global end vertices
  const int32_t* edge_scat;
  const int32_t* edge_off;
  int32_t* cnt;
  int32_t* stats;              // [0] longest row, [1] overflow flag
  const int64_t* rowptr;
  int32_t* col;
};
void launch_mass_pattern(const MassPatternJob& J, bool fill, hipStream_t st);
void launch_csr_to_dense(const int64_t* rowptr, const int32_t* col, const double* val, int n, double* out,
                         int64_t ld, hipStream_t st);
void launch_rebase_i64(const int64_t* in, int64_t n, int64_t* out, hipStream_t st);

struct RhsJob {
  int F, nrhs;
  const double* dirs;          // 3*nrhs
  const double* pols;          // 6*nrhs (re,im per component)
  double k_ext;
  int64_t E_tot;
  double* g;                   // [nrhs][2][E_tot] complex: identity-term projections
  double* h;                   // [nrhs][2][E_tot] complex: L2 projections
};

hipError_t upload_rules(const double* l, const double* w, hipStream_t s);

// Workgroup size of the regular kernel = the most distinct trial triangles a
// chunk of trial edges may hold
int regular_chunk_limit(bool fp64);
template <typename R, typename M>
void launch_regular_rows(const AsmParams<M>& p, const HalfJob<M>& h, int t1_begin, int t1_end, int nchunks,
                         int max_list, hipStream_t st);
// A[rows[r]] += H[sp[r]] + H[sm[r]] (negative slot = absent), complex rows of ncols
template <typename M>
void launch_rows_combine(M* A, int64_t lda, const M* H, int64_t ldh, const int32_t* rows, const int32_t* sp,
                         const int32_t* sm, int nrows, int ncols, hipStream_t st, bool overwrite = false,
                         const int32_t* cstart = nullptr);  // per row: first column written (a multiple of 8)
template <typename M>
void launch_singular(const AsmParams<M>& p, const SingParams& s, hipStream_t st);

// sum of the four slot values of every kept entry, in the order 2a + b
void launch_bc_gather(const BCJob& j, hipStream_t st);
void launch_bc_nearfield(const AsmParams<double>& geo, const CellParams& c, const BCJob& j, hipStream_t st);
void launch_mass(const AsmParams<double>& geo, const CellParams& c, const MassJob& j, hipStream_t st);
void launch_gram(const AsmParams<double>& geo, const MassJob& j, hipStream_t st);
void launch_rhs(const AsmParams<double>& geo, const RhsJob& j, hipStream_t st);

// Linear algebra -------------------------------------------------------------
// Dense PMCHWT block application on a vector batch:
//   yD += C xD + (1/k) S xN ;  yN += -k S xD + C xN
// S, C row-major rows x cols, complex interleaved, element M.  Vectors are
// complex128; vector r of the batch starts at r*vstride.
template <typename M>
void launch_gemv_pmchwt(const M* S, const M* C, int64_t ld, int rows, int cols, double kr, double ki,
                        const double* xD, const double* xN, double* yD, double* yN, int nrhs,
                        int64_t vstride, hipStream_t st);
// One product of a grouped launch: the arguments of launch_gemv_pmchwt for
// nr right-hand sides (1, 2 or 4; the same nr for every job of a launch) and
// the first workgroup of the job (jobs sorted by block0).
template <typename M>
struct GemvJob {
  const M* S;
  const M* C;
  int64_t ld;
  int rows, cols;
  double kr, ki;
  const double* xD;
  const double* xN;
  double* yD;
  double* yN;
  int64_t vstride;
  int block0;
};
// workgroups the product of `rows` rows takes with nr right-hand sides
template <typename M>
int gemv_blocks(int rows, int nr);
template <typename M>
void launch_gemv_pmchwt_grouped(const GemvJob<M>* jobs_dev, int njobs, int nr, int total_blocks, hipStream_t st);
// Single scatterer: the same product from C = Ce + Ci, S1 = Se/ke + Si/ki,
// S2 = -(ke Se + ki Si) (launch_combine3 builds them, n complex entries)
template <typename M>
void launch_gemv_pmchwt3(const M* C, const M* S1, const M* S2, int64_t ld, int rows, int cols, const double* xD,
                         const double* xN, double* yD, double* yN, int nrhs, int64_t vstride, hipStream_t st,
                         bool acc = true);
template <typename M>
void launch_combine3(const M* Se, const M* Ce, const M* Si, const M* Ci, int64_t n, double ke, double kir, double kii,
                     M* C, M* S1, M* S2, hipStream_t st);
// Symmetric-tile form of the same three matrices for one right-hand side:
// upper SYM_T x SYM_T tiles (tij: tile t -> (I, J), I <= J), a CSR correction
// (crow/col: row and column of each entry, rowptr over rows) holding
// X_rc - X_cr where singular pairs make the matrices unsymmetric, and
// nt x nt x SYM_T x 4 doubles of partial sums (nt = ceil(n / SYM_T)).
constexpr int SYM_T = 128;
template <typename M>
void launch_pack_sym3(const M* Se, const M* Ce, const M* Si, const M* Ci, int64_t ld, int n, const int32_t* tij,
                      int64_t ntiles, double ke, double kir, double kii, M* P, hipStream_t st);
template <typename M>
void launch_sym_corr(const M* Se, const M* Ce, const M* Si, const M* Ci, int64_t ld, const int32_t* crow,
                     const int32_t* col, int64_t nnz, double ke, double kir, double kii, M* val, hipStream_t st);
// The same correction from the singular pairs' FP64 local blocks alone (the
// regular contributions to X_rc and X_cr are equal): entry k sums the items
// item[ptr[k]] .. item[ptr[k+1]-1], each (local-block entry << 1 | negate),
// over the blocks (Se, Ce, Si, Ci) of SingParams::blk.
template <typename M>
void launch_sym_corr_sing(const int64_t* ptr, const int32_t* item, const double* blk, int64_t nnz, double ke,
                          double kir, double kii, M* val, hipStream_t st);
// Lower tiles of one dense operator X (n x n, leading dimension ld) from its
// upper tiles, X_rc = X_cr for tile(r) > tile(c), then X_rc += the singular
// asymmetry of operator `op` (0..3 = Se, Ce, Si, Ci) on the correction entries.
template <typename M>
void launch_mirror_lower(M* X, int64_t ld, int n, const int32_t* crow, const int32_t* col, const int64_t* ptr,
                         const int32_t* item, const double* blk, int64_t nnz, int op, hipStream_t st);
template <typename M>
void launch_gemv_sym3(const M* P, const int32_t* tij, int64_t ntiles, int nt, int n, const double* xD,
                      const double* xN, double* part, hipStream_t st);
template <typename M>
void launch_sym_reduce(const double* part, int nt, int n, const int64_t* rowptr, const int32_t* col, const M* val,
                       const double* xD, const double* xN, double* yD, double* yN, hipStream_t st);
// Many right-hand sides on the FP32 matrix cores: same product as
// launch_gemv_pmchwt for FP32 operators with ld a multiple of 16; B1, B2 are
// workspaces of 4 nrhs x 2 ld floats each.
void launch_mfma_pmchwt(const float* S, const float* C, int64_t ld, int rows, int cols, double kr, double ki,
                        const double* xD, const double* xN, double* yD, double* yN, int nrhs, int64_t vstride,
                        float* B1, float* B2, hipStream_t st);
// One scatterer's combined operators C = C^e + C^i, S1 = S^e/k_e + S^i/k_i,
// S2 = -(k_e S^e + k_i S^i) (FP32, ld a multiple of 16) on the matrix cores:
// yD = C xD + S1 xN, yN = C xN + S2 xD (overwritten); BD, BN are workspaces
// of 2 nrhs x 2 ld floats each.
void launch_mfma_comb(const float* C, const float* S1, const float* S2, int64_t ld, int rows, int cols,
                      const double* xD, const double* xN, double* yD, double* yN, int nrhs, int64_t vstride, float* BD,
                      float* BN, hipStream_t st);
// API layout (scatterer-major [D_m ; N_m]) <-> internal layout ([D ; N] over
// the union) of nrhs complex vectors on the device; soff: nsc + 1 edge offsets
void launch_layout(const double* in, double* out, int nrhs, int E, const int32_t* soff, int nsc, bool to_internal,
                   hipStream_t st);
// Block-sparse rows of dense BSR_T x BSR_T FP32 tiles (the sparse operators
// of the preconditioner, for products with many right-hand sides): row tile
// bi holds tiles bptr[bi] .. bptr[bi+1] at column tiles bcol[t]; tiles of a
// real matrix are BSR_T x BSR_T floats, of a complex one BSR_T x 2 BSR_T
// ((re, im) pairs); tiles2 is a second value set on the same pattern (the C
// operator of P) or null.
constexpr int BSR_T = 128;
struct BsrMat {
  int nbr = 0, nbc = 0;
  int64_t ntiles = 0;
  const int64_t* bptr = nullptr;
  const int32_t* bcol = nullptr;
  const float* tiles1 = nullptr;
  const float* tiles2 = nullptr;
};
void launch_bsr_mark(const int64_t* rowptr, const int32_t* col, int n, int nbc, int32_t* flag, hipStream_t st);
void launch_bsr_fill(const int64_t* rowptr, const int32_t* col, const float* val, int n, int nbc, const int32_t* tmap,
                     bool cplx, float* tiles, hipStream_t st);
// y = alpha M x (+ beta y) for a real BSR matrix on both trace components
// (B: 4 nrhs x nbc BSR_T floats)
void launch_bsr_real2(const BsrMat& M, int rows, int cols, double alpha, const double* x, double* y, int nrhs,
                      int64_t vstride, int64_t cstride, float* B, hipStream_t st, bool accumulate = false);
// [yD | yN] += C [xD | xN] + S [xN / k | -k xD] for a complex BSR pair (S in
// tiles1, C in tiles2 or absent); B1, B2: 4 nrhs x 2 nbc BSR_T floats each
void launch_bsr_pmchwt(const BsrMat& M, int rows, int cols, double kr, double ki, const double* xD, const double* xN,
                       double* yD, double* yN, int nrhs, int64_t vstride, float* B1, float* B2, hipStream_t st);
// FP64 matrix-core forms of the two products above (ld a multiple of 8):
// combined operators (BD, BN: 2 nrhs x 2 ld doubles each) and one medium
// (B1, B2: 4 nrhs x 2 ld doubles each, result added to y).
void launch_mfma64_comb(const double* C, const double* S1, const double* S2, int64_t ld, int rows, int cols,
                        const double* xD, const double* xN, double* yD, double* yN, int nrhs, int64_t vstride,
                        double* BD, double* BN, hipStream_t st);
void launch_mfma64_pmchwt(const double* S, const double* C, int64_t ld, int rows, int cols, double kr, double ki,
                          const double* xD, const double* xN, double* yD, double* yN, int nrhs, int64_t vstride,
                          double* B1, double* B2, hipStream_t st);
// y = alpha M x for a real FP32 matrix (ld a multiple of 32, zero padding
// columns) on both trace components, on the matrix cores; B is a workspace
// of 4 nrhs x ld floats.
void launch_mfma_real2(const float* Mat, int64_t ld, int rows, int cols, double alpha, const double* x, double* y,
                       int nrhs, int64_t vstride, int64_t cstride, float* B, hipStream_t st);
// Same with a CSR pattern (rowptr, col) and value arrays S, C (either may be
// null: treated as zero).
template <typename M>
void launch_spmv_pmchwt(const int64_t* rowptr, const int32_t* col, const M* S, const M* C, int rows,
                        double kr, double ki, const double* xD, const double* xN, double* yD, double* yN,
                        int nrhs, int64_t vstride, hipStream_t st, bool acc = true);
// y = alpha * Mreal x (dense real row-major, rows x cols), complex vectors
void launch_gemv_real(const double* Mat, int64_t ld, int rows, int cols, double alpha, const double* x,
                      double* y, int nrhs, int64_t vstride, hipStream_t st);
void launch_transpose(const double* in, double* out, int n, hipStream_t st);
// y = alpha M x for both trace components (second component at +cstride);
// M is double or float (accumulation in double); ld a multiple of 4 with
// zero padding columns
// Truncated CSR copy of an inverse (n x n, row-major, ld): entries of at
// least rel x their row's largest, ascending columns.  build_*: counts (cnt,
// n ints), thresholds (thr, n floats) and rowptr (n + 1); fill_*: col / val of
// rowptr[n] entries.  launch_spmv_real2_csr: the launch_gemv_real2 product
// from that copy.
template <typename T>
void build_truncated_inverse(const T* A, int64_t ld, int n, T rel, int32_t* cnt, T* thr, int64_t* rowptr,
                             hipStream_t st);
template <typename T>
void fill_truncated_inverse(const T* A, int64_t ld, int n, const T* thr, const int64_t* rowptr, int32_t* col, T* val,
                            hipStream_t st);
// One step of the Chebyshev iteration for the inverse of M (n x n; its columns
// as an ELL copy of W slots, entry-major, from launch_csc_to_ell) on X and D
// (n rows, ld); rn_part: one partial sum of ||I - X M||_F^2 per workgroup,
// (n + cheb_rows(n) - 1) / cheb_rows(n) of them.  cheb_width: the ELL width
// for the longest column (0: more than 64 entries)
template <typename T>
int cheb_rows(int n);
int cheb_width(int maxcount);
template <typename T>
void launch_csc_to_ell(const int64_t* colptr, const int32_t* rowidx, const double* val, int n, int W, int32_t* eidx,
                       T* eval, hipStream_t st);
template <typename T>
void launch_cheb_step(T* X, T* D, int64_t ld, int n, const int32_t* eidx, const T* eval, int W, double cD, double cR,
                      double inv_d, bool first, double* rn_part, hipStream_t st);
template <typename T>
void launch_identity_tail(T* X, int64_t ld, int n, hipStream_t st);
// y = alpha A x + beta y (beta = 0: y overwritten) for both components
void launch_spmv_real2_csr(const int64_t* rowptr, const int32_t* col, const float* val, int rows, double alpha,
                           const double* x, double* y, int nrhs, int64_t vstride, int64_t cstride, hipStream_t st,
                           double beta = 0.0);
void launch_spmv_real2_csr(const int64_t* rowptr, const int32_t* col, const double* val, int rows, double alpha,
                           const double* x, double* y, int nrhs, int64_t vstride, int64_t cstride, hipStream_t st,
                           double beta = 0.0);
// The same product for many right-hand sides from a gathered copy of x with
// the right-hand sides adjacent per column (xt: 4 nrhs doubles per column of
// x: xD re, im, xN re, im of each rhs), so that one entry's gathers for a
// group of 4 right-hand sides read 128 contiguous bytes; same sums in the same
// order as launch_spmv_real2_csr.  xt: 4 cols nrhs doubles of workspace.
void launch_spmv_real2_csr_t(const int64_t* rowptr, const int32_t* col, const double* val, int rows, int cols,
                             double alpha, const double* x, double* y, int nrhs, int64_t vstride, int64_t cstride,
                             double* xt, hipStream_t st);
template <typename M>
void launch_gemv_real2(const M* Mat, int64_t ld, int rows, int cols, double alpha, const double* x, double* y,
                       int nrhs, int64_t vstride, int64_t cstride, hipStream_t st);
// n x n row-major (ld n) -> n x n with leading dimension ldo >= n, zero padding
template <typename T>
void launch_repack(const double* in, int n, T* out, int64_t ldo, hipStream_t st);
// blocked Gauss-Jordan inverse helpers (column-major, no pivoting)
void launch_gj_block_inverse(const double* X, int64_t ldx, double* out, int b, hipStream_t st);
void launch_gj_take_columns(double* X, int64_t n, int p0, int b, double* C, hipStream_t st);
// FP32 variants: the block inverse written row-major,
// the taken columns row-major (n x b)
void launch_gj_block_inverse_f32(const float* X, int64_t ldx, float* out_rowmajor, int b, hipStream_t st);
void launch_gj_take_columns_f32(float* X, int64_t n, int p0, int b, float* C, hipStream_t st);
// out (n2 x n2 FP32) = [[in, 0], [0, I]]
void launch_embed_f32(const double* in, int n, float* out, int n2, hipStream_t st);
void launch_transpose_f32(const float* in, float* out, int n, hipStream_t st);
// y (rows x Nr, row stride ldy) = A B^T or y -= A B^T on the FP32 matrix cores;
// A rows x K (stride lda), B Nr x K (stride K), K a multiple of 32
void launch_mfma_f32(const float* A, int64_t lda, const float* B, int K, int rows, int Nr, float* y, int64_t ldy,
                     bool subtract, hipStream_t st);

// GMRES helpers on batches of complex128 vectors of length n.
// w += sign V h; the coefficient (r, i) is the sum of S partial values
// h[(r hstride + i) S + s] (complex), added in order of s.  nrm2 (optional):
// partial sums of |w|^2 of the result, update_blocks(n) per right-hand side
void launch_update(const double* V, int64_t vstep, int nvec, double* w, int64_t wstride, int n,
                   const int32_t* active, int nrhs, int64_t rstride_v, const double* h, int64_t hstride,
                   double sign, hipStream_t st, int S = 1, double* nrm2 = nullptr);
int update_blocks(int n);
// part (optional): scratch of nrhs + 256 doubles for a split reduction
void launch_norms(const double* w, int64_t wstride, int n, int nrhs, double* out, hipStream_t st,
                  double* part = nullptr);
// Split reduction left unfinished: the consumers (launch_update,
// launch_finish_step) add the partial values in order.  Returns S, the
// partials per result: part[((r nvec + i) S + s)] complex, at most
// 2 (1024 + nvec nrhs) doubles.
int dots_splits(int nvec, int nrhs, int n);
int dots_part_only(const double* V, int64_t vstep, int nvec, const double* w, int64_t wstride, int n,
                   const int32_t* active, int nrhs, int64_t rstride_v, double* part, hipStream_t st);
// v = w / sqrt(sum_s nrm2[r S2 + s]) per right-hand side (0 where inactive or
// zero); also the finished sums fin = [h1 | h2 | norms] of the step's two
// projection passes (h1p, h2p: S1 partials per coefficient, nvec coefficients)
// and, once those are visible system-wide, flags[r] = seq (fin and flags may
// be host memory mapped for the device)
void launch_finish_step(const double* w, int64_t wstride, double* v, int64_t vstride, int n, int nrhs,
                        const double* nrm2, int S2, const int32_t* active, const double* h1p, const double* h2p,
                        int S1, int nvec, double* fin, double* flags, double seq, hipStream_t st);
void launch_scale_copy(const double* w, int64_t wstride, double* v, int64_t vstride, int n, int nrhs,
                       const double* scale, hipStream_t st);
// G x = b by conjugate gradients (G: real SPD CSR of n rows; b, x complex,
// per-vector strides in complex entries), one workgroup per vector; work:
// 6 n nvec doubles
void launch_gram_cg(const int64_t* rowptr, const int32_t* col, const double* val, int n, const double* b,
                    int64_t bstride, double* x, int64_t xstride, int nvec, double* work, double tol2, int maxit,
                    hipStream_t st);
void launch_axpby(double* y, const double* x, int64_t stride, int n, int nrhs, double a, double b,
                  hipStream_t st);
// the same on rows [0, rows) of both components (component stride cstride)
void launch_axpby_rows(double* y, const double* x, int64_t vstride, int rows, int64_t cstride, int nrhs, double a,
                       double b, hipStream_t st);
void launch_zero(double* p, int64_t n, hipStream_t st);
void launch_zero_f(float* p, int64_t n, hipStream_t st);
void launch_pack_cols(const double* src, int64_t sstride, int E, int nvec, double* dst, hipStream_t st);
void launch_unpack_cols(const double* src, int E, int nvec, double* dst, int64_t dstride, hipStream_t st);

// Far field: currents on the quadrature points (degree-4 rule, 6 per
// triangle), then a segmented non-uniform Fourier sum.  Workspace sizes (in
// doubles) come from far_field_plan.
struct FarPlan {
  int64_t npts = 0, seg_len = 0;
  int nseg = 1;
  int64_t n_ypts = 0, n_J = 0, n_part = 0;
};
FarPlan far_field_plan(int F, int nrhs, int nobs);
// Far field on the FP64 matrix cores (many right-hand sides): rule points as
// for the VALU sum, the expanded currents B (n_B doubles), K split nsplit
// ways (partial sums part, n_part doubles).
struct FarMfmaPlan {
  int64_t npts = 0;
  int Kt = 0, Nr = 0, nsplit = 1, rows = 0;
  int64_t n_B = 0, n_part = 0;
};
FarMfmaPlan far_mfma_plan(int F, int nrhs, int nobs);
void launch_far_field_mfma(const AsmParams<double>& geo, const double* x, int64_t E_tot, int nrhs, double k,
                           const double* obs, int nobs, double* F_out, const FarMfmaPlan& plan, double* ypts,
                           double* J, double* B, double* part, hipStream_t st);
// The same for nh directions and their antipodes (F_out: 2 nh directions per
// rhs, direction nh + o = -obs[o]): the cosine and sine sums of the currents
// are shared by a direction and its antipode, so the matrix product has half
// the K extent (K = rule points, the currents' real and imaginary parts as
// separate columns).
FarMfmaPlan far_pair_plan(int F, int nrhs, int nh);
void launch_far_field_pair(const AsmParams<double>& geo, const double* x, int64_t E_tot, int nrhs, double k,
                           const double* obs, int nh, double* F_out, const FarMfmaPlan& plan, double* ypts, double* J,
                           double* B, double* part, hipStream_t st);
FarPlan far_field_plan_capped(int F, int nrhs, int nobs, int64_t max_part);
// Total electric field at points (region per point, rule-point data and the
// sums; ypts: 4 doubles per rule point, J: near_j_doubles() per rhs and rule
// point, 6 F rule points)
void launch_near_field(const AsmParams<double>& g, const int32_t* tri_off, int nscat, const double* x,
                       const double* cinc, int64_t E_tot, int nrhs, const double* pts, int npts,
                       const double* dirs, const double* pols, double k_ext, const double* k_int, int32_t* region,
                       double* ypts, double* J, double* Eout, hipStream_t st);
int near_j_doubles();
void launch_far_field(const AsmParams<double>& geo, const double* x, int64_t E_tot, int nrhs, double k,
                      const double* obs, int nobs, double* F_out, const FarPlan& plan, double* ypts, double* J,
                      double* part, hipStream_t st);
void launch_sigma_sca(const double* F, int nobs, int nrhs, const double* w, double* out, hipStream_t st);

// ---------------------------------------------------------------------------
// Geometric classification tables (count pass, scan, fill pass each)
// ---------------------------------------------------------------------------
// uniform grid on the centres of the BC support boxes, cell size h >= chi +
// the largest box extent, so that the 27 cells around a box's own hold every
// box within chi of it
struct NfGrid {
  double gmin[3];
  double h;
  int dims[3];
};
struct NfJob {
  int E;
  const double* box;       // 6 per union edge: lo xyz, hi xyz of the BC support
  const int32_t* escat;    // scatterer of each union edge
  NfGrid g;
  const int32_t* gcell;    // grid cell of each edge
  const int64_t* gstart;   // ncells+1 into gitem
  const int32_t* gitem;    // edges grouped by grid cell
  double chi;
  int cross;               // keep pairs of different scatterers
};
struct CellPairJob {
  const int32_t* inc_ptr;   // ncell+1 into inc_edges (dual cell = primal vertex)
  const int32_t* inc_edges; // union edges incident to each cell, slot order
  const int64_t* rowptr;    // near-field pattern of P
  const int32_t* col;
  const int32_t* ecell;     // 2 per union edge: cells of its end points
  int32_t* ncw;             // count pass: partner cells per cell
  int32_t* nslot;           // count pass: N_v * sum N_w per cell
  int32_t* flag;            // set when a cell has too many partners
  const int64_t* pairoff;   // fill pass: scans of ncw and nslot
  const int64_t* slotbase;
  int32_t* cpairs;          // 2 per pair
  int64_t* slot_off;        // per pair
  int64_t* slot_pos;        // N_v x N_w CSR positions per pair, -1 = cut off
  int64_t* entry_slots;     // 4 per kept entry (i, j): the slot of the cell pair (cell(i, a), cell(j, b)) at 2a + b
};
struct SingListJob {
  int F;
  const int32_t* tvid;     // 3*F vertex ids (global), SoA
  const int32_t* v2t_ptr;  // per global vertex, into v2t
  const int32_t* v2t;      // triangles at each vertex
  int32_t* cnt;            // count pass: pairs per test triangle
  int32_t* flag;           // set when a triangle has too many neighbours
  const int64_t* sptr;     // fill pass: scan of cnt
  int32_t* pairs;          // 2 per pair (test, trial)
  int npts[4];             // Sauter-Schwab points by number of shared vertices
  unsigned long long* point_pairs;
};
struct SymRecJob {
  int64_t npairs;          // singular pairs
  const int32_t* pairs;
  const int32_t* t2e;      // 3*F union edge of local basis a, SoA
  int F, tile, n;          // triangles, tile size, rows (edges)
  int all;                 // every touched entry (no tile filter, no transpose)
  int32_t* cnt;            // records, then entries, per row
  int32_t* maxrec;         // longest record list of a row
  const int64_t* recptr;   // n+1
  int32_t* cur;            // per-row cursor of the record fill
  int64_t* rec;            // (column << 32) | item
  const int64_t* rowptr;   // n+1 entry offsets
  int32_t* crow;
  int32_t* col;
  int64_t* iptr;           // first record of each entry
  int32_t* item;
};
void launch_cls_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st);
void launch_d2f(const double* in, float* out, int64_t n, hipStream_t st);
void launch_cls_set_i64(int64_t* p, int64_t v, hipStream_t st);
void launch_scan_i32(const int32_t* cnt, int n, int64_t* rowptr, hipStream_t st);
void launch_nf_bin(const double* box, int E, const NfGrid& g, int32_t* gcell, int32_t* gcnt, hipStream_t st);
void launch_nf_bin_fill(const int32_t* gcell, int E, const int64_t* gstart, int32_t* gcur, int32_t* gitem,
                        hipStream_t st);
void launch_nf_count(const NfJob& J, int32_t* cnt, int32_t* maxcnt, hipStream_t st);
// cap: a power of two >= the longest row, at most nf_row_capacity()
void launch_nf_fill(const NfJob& J, const int64_t* rowptr, int cap, int32_t* col, hipStream_t st);
void launch_nf_dense(int E, const int32_t* escat, const int32_t* sc_first, const int32_t* sc_n, int cross,
                     int32_t* cnt, int32_t* maxcnt, hipStream_t st);
void launch_nf_dense_fill(int E, const int32_t* escat, const int32_t* sc_first, int cross, const int64_t* rowptr,
                          int32_t* col, hipStream_t st);
void launch_cell_pairs(const CellPairJob& J, int ncell, bool fill, hipStream_t st);
void launch_sing_list(const SingListJob& J, bool fill, hipStream_t st);
void launch_sym_records(const SymRecJob& J, int pass, hipStream_t st);
// cap: a power of two >= the longest record list
void launch_sym_sort(const SymRecJob& J, int cap, hipStream_t st);
void launch_sym_emit(const SymRecJob& J, hipStream_t st);
void launch_count_regular(int F, const double* tcen, const double* tdiam2, const int32_t* tvid, int n_near,
                          int n_medium, int n_far, unsigned long long* out, hipStream_t st);
int cell_pair_capacity();
int nf_row_capacity();
int sing_neighbour_capacity();

}  // namespace pmchwt
