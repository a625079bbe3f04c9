// PMCHWT operator product for many right-hand sides on the FP32 matrix cores
// (the block product of Section 3.2 applied to all incident fields at once).
//
// For one medium,  [Y_D | Y_N] = C [X_D | X_N] + S [X_N / k | -k X_D]
// (Y_D = C X_D + (1/k) S X_N,  Y_N = -k S X_D + C X_N).
// The complex product is one real GEMM: an operator stored as interleaved
// (re, im) FP32 pairs is read as a real matrix Ahat (rows x 2 ld), and every
// complex entry b of the right-hand block becomes the real 2 x 2 block
// [[Re b, Im b], [-Im b, Re b]] of Bhat, so that column 2c of Ahat Bhat is
// Re(A b_c) and column 2c + 1 is Im(A b_c) -- the interleaved complex result,
// at the flop count of the complex product (8 real flops per complex MAC).
// Bhat is stored transposed (real columns x K, K contiguous) so that both
// operands stream along K.
#include "common.hpp"
#include "kernels.hpp"

namespace pmchwt {

typedef float mf4 __attribute__((ext_vector_type(4)));
typedef float mf16 __attribute__((ext_vector_type(16)));

constexpr int MF_BM = 128, MF_BN = 128, MF_BK = 32, MF_LDK = MF_BK + 4;

// Bhat^T for C (B1) and S (B2): real row 2c / 2c+1 for complex column c of
// the right-hand block (c < n: D part of rhs c, else N part of rhs c - n);
// real column 2k / 2k+1 for complex row k (zero for k >= E).
__global__ void k_mfma_rhs(const double* __restrict__ xD, const double* __restrict__ xN, int64_t vstride, int E,
                           int Kt, int nrhs, double kr, double ki, float* __restrict__ B1, float* __restrict__ B2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;  // complex row
  const int c = blockIdx.y;                             // complex column
  if (2 * k >= Kt) return;
  double b1r = 0, b1i = 0, b2r = 0, b2i = 0;
  if (k < E) {
    const double k2 = kr * kr + ki * ki;
    const double ikr = kr / k2, iki = -ki / k2;  // 1/k
    if (c < nrhs) {
      const double* d = xD + 2 * (int64_t(c) * vstride + k);
      const double* n = xN + 2 * (int64_t(c) * vstride + k);
      b1r = d[0];
      b1i = d[1];
      b2r = n[0] * ikr - n[1] * iki;  // xN / k
      b2i = n[0] * iki + n[1] * ikr;
    } else {
      const double* d = xD + 2 * (int64_t(c - nrhs) * vstride + k);
      const double* n = xN + 2 * (int64_t(c - nrhs) * vstride + k);
      b1r = n[0];
      b1i = n[1];
      b2r = -(kr * d[0] - ki * d[1]);  // -k xD
      b2i = -(kr * d[1] + ki * d[0]);
    }
  }
  const int64_t r0 = int64_t(2 * c) * Kt + 2 * k, r1 = r0 + Kt;
  B1[r0] = float(b1r);
  B1[r0 + 1] = float(-b1i);
  B1[r1] = float(b1i);
  B1[r1 + 1] = float(b1r);
  B2[r0] = float(b2r);
  B2[r0 + 1] = float(-b2i);
  B2[r1] = float(b2i);
  B2[r1 + 1] = float(b2r);
}

// Bhat^T of a plain complex block X (nrhs columns, vectors vstride apart):
// real row 2c / 2c+1 for column c, real column 2k / 2k+1 for complex row k
// (zero for k >= E), the 2 x 2 real block of every complex entry.
template <typename T>
__global__ void k_mfma_rhs_plain(const double* __restrict__ x, int64_t vstride, int E, int Kt, T* __restrict__ B) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;  // complex row
  const int c = blockIdx.y;                             // complex column
  if (2 * k >= Kt) return;
  double br = 0, bi = 0;
  if (k < E) {
    br = x[2 * (int64_t(c) * vstride + k)];
    bi = x[2 * (int64_t(c) * vstride + k) + 1];
  }
  const int64_t r0 = int64_t(2 * c) * Kt + 2 * k, r1 = r0 + Kt;
  B[r0] = T(br);
  B[r0 + 1] = T(-bi);
  B[r1] = T(bi);
  B[r1 + 1] = T(br);
}

// Output mappings of the real GEMM columns.
// Complex block: real column n -> complex column n/2, part n%2 (overwrites y).
template <typename R>
struct CplxOut {
  static constexpr bool kInit = false, kNegA = false;
  __device__ __forceinline__ R init(int, int) const { return R(0); }
  double* y;
  int64_t vstride;
  __device__ __forceinline__ void put(int r, int n, R v) const {
    y[2 * (int64_t(n >> 1) * vstride + r) + (n & 1)] = double(v);
  }
};
// PMCHWT product: real column n -> complex column c = n/2, part n%2;
// c < nrhs -> yD of rhs c, else yN of rhs c - nrhs; added to y.
struct PmchwtOut {
  static constexpr bool kInit = false, kNegA = false;
  __device__ __forceinline__ float init(int, int) const { return 0.0f; }
  double* yD;
  double* yN;
  int64_t vstride;
  int nrhs;
  __device__ __forceinline__ void put(int r, int n, float v) const {
    const int cc = n >> 1, part = n & 1;
    double* base = cc < nrhs ? yD + 2 * int64_t(cc) * vstride : yN + 2 * int64_t(cc - nrhs) * vstride;
    base[2 * int64_t(r) + part] += double(v);
  }
};
// Real matrix on complex vectors of two trace components: real column n ->
// rhs n/4, component (n/2)%2 (second at +cstride), part n%2; y = alpha M x.
struct Real2Out {
  static constexpr bool kInit = false, kNegA = false;
  __device__ __forceinline__ float init(int, int) const { return 0.0f; }
  double* y;
  int64_t vstride, cstride;
  double alpha;
  __device__ __forceinline__ void put(int r, int n, float v) const {
    const int q = n >> 2, comp = (n >> 1) & 1, part = n & 1;
    y[2 * (int64_t(q) * vstride + comp * cstride + r) + part] = alpha * double(v);
  }
};

// The same, added: y = alpha M x + y.
struct Real2AccOut {
  static constexpr bool kInit = false, kNegA = false;
  __device__ __forceinline__ float init(int, int) const { return 0.0f; }
  double* y;
  int64_t vstride, cstride;
  double alpha;
  __device__ __forceinline__ void put(int r, int n, float v) const {
    const int q = n >> 2, comp = (n >> 1) & 1, part = n & 1;
    y[2 * (int64_t(q) * vstride + comp * cstride + r) + part] += alpha * double(v);
  }
};

// Plain FP32 matrices: y[r * ld + n] = v, or y[r * ld + n] -= v.
// (kInit: the accumulators start from init(r, n), and with kNegA the
// product enters with a minus sign, so that y -= A B^T ends in plain stores)
struct StoreOut {
  static constexpr bool kInit = false, kNegA = false;
  float* y;
  int64_t ld;
  __device__ __forceinline__ float init(int, int) const { return 0.0f; }
  __device__ __forceinline__ void put(int r, int n, float v) const { y[int64_t(r) * ld + n] = v; }
};
struct SubOut {
  static constexpr bool kInit = true, kNegA = true;
  float* y;
  int64_t ld;
  __device__ __forceinline__ float init(int r, int n) const { return y[int64_t(r) * ld + n]; }
  __device__ __forceinline__ void put(int r, int n, float v) const { y[int64_t(r) * ld + n] = v; }
};

// out(rows x Nr) = A1 B1^T (K1) + A2 B2^T (K2), K1 and K2 multiples of 32
// (K2 = 0 for a single product); B rows have stride K.
// Workgroup tile 128 x 128, four wavefronts of 64 x 64 = 2 x 2 MFMA 32x32x2
// tiles; K tiles of 32 double-buffered in LDS (rows padded to 36 floats),
// the next tile prefetched into registers during the MFMAs.  Each lane feeds
// the MFMA k-slot (lane / 32) with k = 16 (lane / 32) + step, the same
// permutation of k for both operands, so its 16 values per tile are
// contiguous in LDS.
template <typename Out>
__device__ __forceinline__ void mfma_gemm_tile(const float* __restrict__ A1, const float* __restrict__ B1, int K1,
                                               int64_t lda1, const float* __restrict__ A2,
                                               const float* __restrict__ B2, int K2, int64_t lda2, int rows, int Nr,
                                               const Out& out) {
  __shared__ float As[2][MF_BM * MF_LDK];
  __shared__ float Bs[2][MF_BN * MF_LDK];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = blockIdx.y * MF_BM, n0 = blockIdx.x * MF_BN;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
  const int h = lane >> 5, l32 = lane & 31;
  mf16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc[i][j] = mf16{};
      if constexpr (Out::kInit) {
        const int n = n0 + wc + 32 * j + l32;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int r = m0 + wr + 32 * i + 8 * (e >> 2) + 4 * h + (e & 3);
          if (r < rows && n < Nr) acc[i][j][e] = out.init(r, n);
        }
      }
    }
  const int lr = t >> 3, lc = (t & 7) * 4;
  const int nt1 = K1 / MF_BK, nt = nt1 + K2 / MF_BK;
  mf4 ra[4], rb[4];
  auto gload = [&](int kt) {
    const bool first = kt < nt1;
    const float* A = first ? A1 : A2;
    const float* B = first ? B1 : B2;
    const int64_t la = first ? lda1 : lda2;
    const int kb = first ? K1 : K2;
    const int k0 = (first ? kt : kt - nt1) * MF_BK;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = min(m0 + lr + 32 * q, rows - 1), c = min(n0 + lr + 32 * q, Nr - 1);
      ra[q] = __builtin_nontemporal_load(reinterpret_cast<const mf4*>(A + int64_t(r) * la + k0 + lc));
      rb[q] = *reinterpret_cast<const mf4*>(B + int64_t(c) * kb + k0 + lc);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      *reinterpret_cast<mf4*>(&As[buf][(lr + 32 * q) * MF_LDK + lc]) = ra[q];
      *reinterpret_cast<mf4*>(&Bs[buf][(lr + 32 * q) * MF_LDK + lc]) = rb[q];
    }
  };
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nt; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nt) gload(kt + 1);
    float af[2][16], bf[2][16];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        mf4 a = *reinterpret_cast<const mf4*>(&As[buf][(wr + 32 * i + l32) * MF_LDK + 16 * h + 4 * q]);
        const mf4 b = *reinterpret_cast<const mf4*>(&Bs[buf][(wc + 32 * i + l32) * MF_LDK + 16 * h + 4 * q]);
        if constexpr (Out::kNegA) a = -a;
        af[i][4 * q] = a.x;
        af[i][4 * q + 1] = a.y;
        af[i][4 * q + 2] = a.z;
        af[i][4 * q + 3] = a.w;
        bf[i][4 * q] = b.x;
        bf[i][4 * q + 1] = b.y;
        bf[i][4 * q + 2] = b.z;
        bf[i][4 * q + 3] = b.w;
      }
#pragma unroll
    for (int kk = 0; kk < 16; ++kk)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i][kk], bf[j][kk], acc[i][j], 0, 0, 0);
    if (kt + 1 < nt) sstore(buf ^ 1);
    __syncthreads();
  }
  // epilogue: 32x32 accumulator element e of lane l is row 8 (e/4) + 4 (l/32) + e%4, column l%32
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wc + 32 * j + l32;
      if (n >= Nr) continue;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int r = m0 + wr + 32 * i + 8 * (e >> 2) + 4 * h + (e & 3);
        if (r < rows) out.put(r, n, acc[i][j][e]);
      }
    }
}

template <typename Out>
__global__ __launch_bounds__(256, 2) void k_mfma_gemm(const float* __restrict__ A1, const float* __restrict__ B1,
                                                      int K1, int64_t lda1, const float* __restrict__ A2,
                                                      const float* __restrict__ B2, int K2, int64_t lda2, int rows,
                                                      int Nr, Out out) {
  mfma_gemm_tile<Out>(A1, B1, K1, lda1, A2, B2, K2, lda2, rows, Nr, out);
}

// Two products of the same shape in one launch, blockIdx.z picking (a) or
// (b) (selected in scalar registers): twice the workgroups of one product
// for outputs whose tiles alone do not fill the chip.
template <typename Out>
__global__ __launch_bounds__(256, 2) void k_mfma_gemm2(const float* A1a, const float* B1a, const float* A2a,
                                                       const float* B2a, Out oa, const float* A1b, const float* B1b,
                                                       const float* A2b, const float* B2b, Out ob, int K, int64_t lda,
                                                       int rows, int Nr) {
  const bool zb = blockIdx.z != 0;
  const Out out = zb ? ob : oa;
  mfma_gemm_tile<Out>(zb ? A1b : A1a, zb ? B1b : B1a, K, lda, zb ? A2b : A2a, zb ? B2b : B2a, K, lda, rows, Nr, out);
}

// Xhat^T for a real matrix: row n = (rhs n/4, component (n/2)%2, part n%2),
// column k < E the value, zero up to Kt.
__global__ void k_mfma_rhs_real(const double* __restrict__ x, int64_t vstride, int64_t cstride, int E, int Kt,
                                int nrhs, float* __restrict__ B) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = blockIdx.y;
  if (k >= Kt) return;
  const int q = n >> 2, comp = (n >> 1) & 1, part = n & 1;
  B[int64_t(n) * Kt + k] = k < E ? float(x[2 * (int64_t(q) * vstride + comp * cstride + k) + part]) : 0.0f;
}

void launch_mfma_f32(const float* A, int64_t lda, const float* B, int K, int rows, int Nr, float* y, int64_t ldy,
                     bool subtract, hipStream_t st) {
  const dim3 grid(unsigned((Nr + MF_BN - 1) / MF_BN), unsigned((rows + MF_BM - 1) / MF_BM));
  if (subtract)
    hipLaunchKernelGGL((k_mfma_gemm<SubOut>), grid, dim3(256), 0, st, A, B, K, lda, A, B, 0, lda, rows, Nr,
                       SubOut{y, ldy});
  else
    hipLaunchKernelGGL((k_mfma_gemm<StoreOut>), grid, dim3(256), 0, st, A, B, K, lda, A, B, 0, lda, rows, Nr,
                       StoreOut{y, ldy});
}

void launch_mfma_real2(const float* Mat, int64_t ld, int rows, int cols, double alpha, const double* x, double* y,
                       int nrhs, int64_t vstride, int64_t cstride, float* B, hipStream_t st) {
  const int Kt = int(ld);  // a multiple of 32
  const int Nr = 4 * nrhs;
  hipLaunchKernelGGL(k_mfma_rhs_real, dim3(unsigned((Kt + 255) / 256), unsigned(Nr)), dim3(256), 0, st, x, vstride,
                     cstride, cols, Kt, nrhs, B);
  const dim3 grid(unsigned((Nr + MF_BN - 1) / MF_BN), unsigned((rows + MF_BM - 1) / MF_BM));
  hipLaunchKernelGGL((k_mfma_gemm<Real2Out>), grid, dim3(256), 0, st, Mat, B, Kt, ld, Mat, B, 0, ld, rows, Nr,
                     Real2Out{y, vstride, cstride, alpha});
}

void launch_mfma_pmchwt(const float* S, const float* C, int64_t ld, int rows, int cols, double kr, double ki,
                        const double* xD, const double* xN, double* yD, double* yN, int nrhs, int64_t vstride,
                        float* B1, float* B2, hipStream_t st) {
  const int Kt = int(2 * ld);  // real K per operand (ld is a multiple of 16)
  const int Nr = 4 * nrhs;     // real columns
  hipLaunchKernelGGL(k_mfma_rhs, dim3(unsigned((Kt / 2 + 255) / 256), unsigned(2 * nrhs)), dim3(256), 0, st, xD, xN,
                     vstride, cols, Kt, nrhs, kr, ki, B1, B2);
  const dim3 grid(unsigned((Nr + MF_BN - 1) / MF_BN), unsigned((rows + MF_BM - 1) / MF_BM));
  hipLaunchKernelGGL((k_mfma_gemm<PmchwtOut>), grid, dim3(256), 0, st, C, B1, Kt, 2 * ld, S, B2, Kt, 2 * ld, rows, Nr,
                     PmchwtOut{yD, yN, vstride, nrhs});
}

// ---------------------------------------------------------------------------
// Sparse operators (the near-field P, the sparse mass inverses) applied to
// many right-hand sides on the matrix cores, as block-sparse rows of dense
// 128 x 128 tiles: a product with a tile reuses each loaded right-hand-side
// value for 128 rows, where a CSR product gathers it once per entry.
// ---------------------------------------------------------------------------

// flag[(i / BSR_T) nbc + col / BSR_T] = 1 for every entry of rows [0, n)
__global__ void k_bsr_mark(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col, int n, int nbc,
                           int32_t* __restrict__ flag) {
  const int i = blockIdx.x;
  if (i >= n) return;
  for (int64_t e = rowptr[i] + threadIdx.x; e < rowptr[i + 1]; e += blockDim.x)
    flag[int64_t(i / BSR_T) * nbc + col[e] / BSR_T] = 1;
}

// tile values (zeroed beforehand): entry (i, j) of tile tmap[(i / T) nbc + j / T]
// at row i % T, real column j % T (cplx: 2 (j % T) + {re, im})
template <bool CPLX>
__global__ void k_bsr_fill(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                           const float* __restrict__ val, int n, int nbc, const int32_t* __restrict__ tmap,
                           float* __restrict__ tiles) {
  const int i = blockIdx.x;
  if (i >= n) return;
  constexpr int KW = CPLX ? 2 * BSR_T : BSR_T;
  const int64_t rb = int64_t(i / BSR_T) * nbc;
  for (int64_t e = rowptr[i] + threadIdx.x; e < rowptr[i + 1]; e += blockDim.x) {
    const int j = col[e];
    float* t = tiles + int64_t(tmap[rb + j / BSR_T]) * BSR_T * KW + int64_t(i % BSR_T) * KW;
    if (CPLX) {
      t[2 * (j % BSR_T)] = val[2 * e];
      t[2 * (j % BSR_T) + 1] = val[2 * e + 1];
    } else {
      t[j % BSR_T] = val[e];
    }
  }
}

void launch_bsr_mark(const int64_t* rowptr, const int32_t* col, int n, int nbc, int32_t* flag, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_bsr_mark, dim3(unsigned(n)), dim3(64), 0, st, rowptr, col, n, nbc, flag);
}
void launch_bsr_fill(const int64_t* rowptr, const int32_t* col, const float* val, int n, int nbc, const int32_t* tmap,
                     bool cplx, float* tiles, hipStream_t st) {
  if (n <= 0) return;
  if (cplx)
    hipLaunchKernelGGL(k_bsr_fill<true>, dim3(unsigned(n)), dim3(64), 0, st, rowptr, col, val, n, nbc, tmap, tiles);
  else
    hipLaunchKernelGGL(k_bsr_fill<false>, dim3(unsigned(n)), dim3(64), 0, st, rowptr, col, val, n, nbc, tmap, tiles);
}

// out = V1 B1 (+ V2 B2) over the tiles of the workgroup's row tile: tiles of
// KW real columns (KW = 128 real, 256 complex as (re, im) pairs), the tile
// in row-tile list position t at real K offset bcol[t] KW of the B rows
// (length Kt).  Same MFMA tiling, LDS layout and prefetch as k_mfma_gemm.
template <typename Out>
__global__ __launch_bounds__(256, 2) void k_mfma_bsr(const float* __restrict__ V1, const float* __restrict__ V2,
                                                     const int64_t* __restrict__ bptr,
                                                     const int32_t* __restrict__ bcol, int KW,
                                                     const float* __restrict__ B1, const float* __restrict__ B2,
                                                     int Kt, int rows, int Nr, Out out) {
  __shared__ float As[2][MF_BM * MF_LDK];
  __shared__ float Bs[2][MF_BN * MF_LDK];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int bi = blockIdx.y;
  const int m0 = bi * MF_BM, n0 = blockIdx.x * MF_BN;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
  const int h = lane >> 5, l32 = lane & 31;
  mf16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = mf16{};
  const int64_t tb = bptr[bi];
  const int ntl = int(bptr[bi + 1] - tb), kpt = KW / MF_BK;
  const int nseg = V2 ? 2 : 1, nt = nseg * ntl * kpt;
  const int lr = t >> 3, lc = (t & 7) * 4;
  mf4 ra[4], rb[4];
  auto gload = [&](int kt) {
    const int seg = kt / (ntl * kpt), rem = kt - seg * ntl * kpt, tl = rem / kpt, kk = rem - tl * kpt;
    const float* A = (seg == 0 ? V1 : V2) + (tb + tl) * int64_t(BSR_T) * KW + kk * MF_BK + lc;
    const float* B = (seg == 0 ? B1 : B2) + int64_t(bcol[tb + tl]) * KW + kk * MF_BK + lc;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = min(n0 + lr + 32 * q, Nr - 1);
      ra[q] = __builtin_nontemporal_load(reinterpret_cast<const mf4*>(A + int64_t(lr + 32 * q) * KW));
      rb[q] = *reinterpret_cast<const mf4*>(B + int64_t(c) * Kt);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      *reinterpret_cast<mf4*>(&As[buf][(lr + 32 * q) * MF_LDK + lc]) = ra[q];
      *reinterpret_cast<mf4*>(&Bs[buf][(lr + 32 * q) * MF_LDK + lc]) = rb[q];
    }
  };
  if (nt > 0) {
    gload(0);
    sstore(0);
  }
  __syncthreads();
  for (int kt = 0; kt < nt; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nt) gload(kt + 1);
    float af[2][16], bf[2][16];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const mf4 a = *reinterpret_cast<const mf4*>(&As[buf][(wr + 32 * i + l32) * MF_LDK + 16 * h + 4 * q]);
        const mf4 b = *reinterpret_cast<const mf4*>(&Bs[buf][(wc + 32 * i + l32) * MF_LDK + 16 * h + 4 * q]);
        af[i][4 * q] = a.x;
        af[i][4 * q + 1] = a.y;
        af[i][4 * q + 2] = a.z;
        af[i][4 * q + 3] = a.w;
        bf[i][4 * q] = b.x;
        bf[i][4 * q + 1] = b.y;
        bf[i][4 * q + 2] = b.z;
        bf[i][4 * q + 3] = b.w;
      }
#pragma unroll
    for (int kk = 0; kk < 16; ++kk)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i][kk], bf[j][kk], acc[i][j], 0, 0, 0);
    if (kt + 1 < nt) sstore(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wc + 32 * j + l32;
      if (n >= Nr) continue;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int r = m0 + wr + 32 * i + 8 * (e >> 2) + 4 * h + (e & 3);
        if (r < rows) out.put(r, n, acc[i][j][e]);
      }
    }
}

void launch_bsr_real2(const BsrMat& M, int rows, int cols, double alpha, const double* x, double* y, int nrhs,
                      int64_t vstride, int64_t cstride, float* B, hipStream_t st, bool accumulate) {
  const int Kt = M.nbc * BSR_T;
  const int Nr = 4 * nrhs;
  hipLaunchKernelGGL(k_mfma_rhs_real, dim3(unsigned((Kt + 255) / 256), unsigned(Nr)), dim3(256), 0, st, x, vstride,
                     cstride, cols, Kt, nrhs, B);
  const dim3 grid(unsigned((Nr + MF_BN - 1) / MF_BN), unsigned(M.nbr));
  const float* none = nullptr;
  if (accumulate)
    hipLaunchKernelGGL((k_mfma_bsr<Real2AccOut>), grid, dim3(256), 0, st, M.tiles1, none, M.bptr, M.bcol, BSR_T, B, B,
                       Kt, rows, Nr, Real2AccOut{y, vstride, cstride, alpha});
  else
    hipLaunchKernelGGL((k_mfma_bsr<Real2Out>), grid, dim3(256), 0, st, M.tiles1, none, M.bptr, M.bcol, BSR_T, B, B, Kt,
                       rows, Nr, Real2Out{y, vstride, cstride, alpha});
}

void launch_bsr_pmchwt(const BsrMat& M, int rows, int cols, double kr, double ki, const double* xD, const double* xN,
                       double* yD, double* yN, int nrhs, int64_t vstride, float* B1, float* B2, hipStream_t st) {
  const int Kt = M.nbc * 2 * BSR_T;
  const int Nr = 4 * nrhs;
  hipLaunchKernelGGL(k_mfma_rhs, dim3(unsigned((Kt / 2 + 255) / 256), unsigned(2 * nrhs)), dim3(256), 0, st, xD, xN,
                     vstride, cols, Kt, nrhs, kr, ki, B1, B2);
  const dim3 grid(unsigned((Nr + MF_BN - 1) / MF_BN), unsigned(M.nbr));
  // C (tiles2, may be absent) against B1 = [X_D | X_N], S (tiles1) against B2
  if (M.tiles2)
    hipLaunchKernelGGL((k_mfma_bsr<PmchwtOut>), grid, dim3(256), 0, st, M.tiles2, M.tiles1, M.bptr, M.bcol,
                       2 * BSR_T, B1, B2, Kt, rows, Nr, PmchwtOut{yD, yN, vstride, nrhs});
  else
    hipLaunchKernelGGL((k_mfma_bsr<PmchwtOut>), grid, dim3(256), 0, st, M.tiles1, static_cast<const float*>(nullptr),
                       M.bptr, M.bcol, 2 * BSR_T, B2, B2, Kt, rows, Nr, PmchwtOut{yD, yN, vstride, nrhs});
}

// One scatterer, the three combined operators C, S1, S2 (FP32, ld a multiple
// of 16): yD = C xD + S1 xN and yN = C xN + S2 xD, two GEMMs of two K
// segments each in one launch (four complex products per right-hand side
// instead of the eight of the per-medium form).  BD, BN: workspaces of 2 nrhs x 2 ld floats.
void launch_mfma_comb(const float* C, const float* S1, const float* S2, int64_t ld, int rows, int cols,
                      const double* xD, const double* xN, double* yD, double* yN, int nrhs, int64_t vstride, float* BD,
                      float* BN, hipStream_t st) {
  const int Kt = int(2 * ld);
  const int Nr = 2 * nrhs;
  const dim3 gb(unsigned((Kt / 2 + 255) / 256), unsigned(nrhs));
  hipLaunchKernelGGL(k_mfma_rhs_plain<float>, gb, dim3(256), 0, st, xD, vstride, cols, Kt, BD);
  hipLaunchKernelGGL(k_mfma_rhs_plain<float>, gb, dim3(256), 0, st, xN, vstride, cols, Kt, BN);
  const dim3 grid(unsigned((Nr + MF_BN - 1) / MF_BN), unsigned((rows + MF_BM - 1) / MF_BM), 2);
  hipLaunchKernelGGL((k_mfma_gemm2<CplxOut<float>>), grid, dim3(256), 0, st, C, BD, S1, BN, CplxOut<float>{yD, vstride},
                     C, BN, S2, BD, CplxOut<float>{yN, vstride}, Kt, 2 * ld, rows, Nr);
}

}  // namespace pmchwt
