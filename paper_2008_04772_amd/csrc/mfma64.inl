// FP64 products on the matrix cores (v_mfma_f64_16x16x4f64): the PMCHWT
// block product of Section 3.2 for many right-hand sides in FP64, and the
// far-field sum of the Stratton-Chu representation (Section 2) as a complex
// matrix product between the plane-wave phases and the surface currents.
//
// Complex products are real GEMMs as in the FP32 kernel: the left operand is
// read as interleaved (re, im) pairs, every complex entry of the right
// operand becomes the real 2 x 2 block [[Re b, Im b], [-Im b, Re b]] of Bhat,
// stored transposed (real columns x K, K contiguous).
//
// Workgroup tile 128 x 128 (four wavefronts of 64 x 64 = 4 x 4 MFMA tiles of
// 16 x 16), K tiles of 16 doubles double-buffered in LDS, k-major there
// ([k][row], rows padded) so that the sixteen lanes of one MFMA k-slot read
// sixteen consecutive doubles; the next K tile is loaded into registers
// during the MFMAs.  MFMA operand layout: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16] of a 16 x 4 by 4 x 16 step; accumulator element v of
// lane l is D[l / 16 + 4 v][l % 16] (measured with one-hot operands).
#include "common.hpp"
#include "kernels.hpp"

namespace pmchwt {

typedef double md4 __attribute__((ext_vector_type(4)));
typedef double md2 __attribute__((ext_vector_type(2)));

constexpr int M64_BM = 128, M64_BN = 128, M64_BK = 16, M64_LD = M64_BM + 2;

// Left operand in memory: up to two K segments (A1 with B1, then A2 with B2),
// row-major with leading dimensions lda1 / lda2; B rows have stride K1 / K2.
struct Mem2Src {
  const double* A1;
  const double* B1;
  int K1;
  int64_t lda1;
  const double* A2;
  const double* B2;
  int K2;
  int64_t lda2;
  static constexpr bool A_PAIRS = false;
  __device__ __forceinline__ int ntiles() const { return (K1 + K2) / M64_BK; }
  // thread t: row t / 2, eight doubles from column 8 (t % 2) of the tile
  __device__ __forceinline__ void load(int kt, int m0, int n0, int rows, int Nr, int t, double (&ra)[8],
                                       double (&rb)[8]) const {
    const int nt1 = K1 / M64_BK;
    const bool first = kt < nt1;
    const double* A = first ? A1 : A2;
    const double* B = first ? B1 : B2;
    const int64_t la = first ? lda1 : lda2;
    const int kb = first ? K1 : K2;
    const int k0 = (first ? kt : kt - nt1) * M64_BK + 8 * (t & 1);
    const int r = min(m0 + (t >> 1), rows - 1), c = min(n0 + (t >> 1), Nr - 1);
    const md2* pa = reinterpret_cast<const md2*>(A + int64_t(r) * la + k0);
    const md2* pb = reinterpret_cast<const md2*>(B + int64_t(c) * kb + k0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const md2 a = __builtin_nontemporal_load(pa + q);
      const md2 b = pb[q];
      ra[2 * q] = a.x;
      ra[2 * q + 1] = a.y;
      rb[2 * q] = b.x;
      rb[2 * q + 1] = b.y;
    }
  }
};

// Left operand generated: Ahat[o][2p + {0, 1}] = (cos, sin) of -k xh_o . y_p
// (the phases of the far-field sum); split z = blockIdx.z of nsplit takes the
// K tiles [z nkt / nsplit, (z + 1) nkt / nsplit).  B (the expanded weighted
// currents) in memory.
struct FarSrc {
  const double* obs;   // 3 per direction
  const double* ypts;  // 4 per rule point
  const double* B;     // Nr x Kt
  int64_t npts;
  int Kt, nobs;
  double k;
  int nkt, nsplit;
  static constexpr bool A_PAIRS = false;
  __device__ __forceinline__ int kt0() const { return int(int64_t(blockIdx.z) * nkt / nsplit); }
  __device__ __forceinline__ int ntiles() const { return int(int64_t(blockIdx.z + 1) * nkt / nsplit) - kt0(); }
  __device__ __forceinline__ void load(int kt, int m0, int n0, int rows, int Nr, int t, double (&ra)[8],
                                       double (&rb)[8]) const {
    const int k0 = (kt0() + kt) * M64_BK + 8 * (t & 1);
    const int o = min(m0 + (t >> 1), rows - 1), c = min(n0 + (t >> 1), Nr - 1);
    const double xh0 = -k * obs[3 * o], xh1 = -k * obs[3 * o + 1], xh2 = -k * obs[3 * o + 2];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t p = min<int64_t>((k0 >> 1) + q, npts - 1);  // padding columns meet zero rows of B
      const double* y = ypts + 4 * p;
      double sn, cs;
      sincos_taylor(xh0 * y[0] + xh1 * y[1] + xh2 * y[2], &sn, &cs);
      ra[2 * q] = cs;
      ra[2 * q + 1] = sn;
    }
    const double2* pb = reinterpret_cast<const double2*>(B + int64_t(c) * Kt + k0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double2 b = pb[q];
      rb[2 * q] = b.x;
      rb[2 * q + 1] = b.y;
    }
  }
};

// Antipodal pairs: a 128-row tile holds 64 directions, their cosine rows
// (0..63) then their sine rows (64..127), of -k xh_o . y_p; K runs over the
// rule points (K tile = 16 points) and B (Nr x Kt) holds the real and the
// imaginary part of each complex current column as two real columns.  Thread
// t computes the four points 4 (t % 4) + j of direction t / 4 once and
// supplies both rows (A_PAIRS: ra[2 j] = cos, ra[2 j + 1] = sin).
struct FarPairSrc {
  const double* obs;   // 3 per direction
  const double* ypts;  // 4 per rule point
  const double* B;     // Nr x Kt
  int64_t npts;
  int Kt, nh;
  double k;
  int nkt, nsplit;
  static constexpr bool A_PAIRS = true;
  __device__ __forceinline__ int kt0() const { return int(int64_t(blockIdx.z) * nkt / nsplit); }
  __device__ __forceinline__ int ntiles() const { return int(int64_t(blockIdx.z + 1) * nkt / nsplit) - kt0(); }
  __device__ __forceinline__ void load(int kt, int m0, int n0, int, int Nr, int t, double (&ra)[8],
                                       double (&rb)[8]) const {
    const int kb = (kt0() + kt) * M64_BK;
    const int o = min((m0 >> 1) + (t >> 2), nh - 1);
    const double xh0 = -k * obs[3 * o], xh1 = -k * obs[3 * o + 1], xh2 = -k * obs[3 * o + 2];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t p = min<int64_t>(kb + 4 * (t & 3) + j, npts - 1);  // padding points meet zero rows of B
      const double* y = ypts + 4 * p;
      double sn, cs;
      sincos_taylor(xh0 * y[0] + xh1 * y[1] + xh2 * y[2], &sn, &cs);
      ra[2 * j] = cs;
      ra[2 * j + 1] = sn;
    }
    const int c = min(n0 + (t >> 1), Nr - 1);
    const double2* pb = reinterpret_cast<const double2*>(B + int64_t(c) * Kt + kb + 8 * (t & 1));
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double2 b = pb[q];
      rb[2 * q] = b.x;
      rb[2 * q + 1] = b.y;
    }
  }
};

// Output mappings.  Complex block (real column n -> complex column n / 2,
// part n % 2; overwrites y).
struct Cplx64Out {
  double* y;
  int64_t vstride;
  __device__ __forceinline__ void put(int r, int n, int, double v) const {
    y[2 * (int64_t(n >> 1) * vstride + r) + (n & 1)] = v;
  }
};
// PMCHWT product of one medium: complex column c < nrhs -> yD of rhs c, else
// yN of rhs c - nrhs; added to y.
struct Pmchwt64Out {
  double* yD;
  double* yN;
  int64_t vstride;
  int nrhs;
  __device__ __forceinline__ void put(int r, int n, int, double v) const {
    const int cc = n >> 1;
    double* base = cc < nrhs ? yD + 2 * int64_t(cc) * vstride : yN + 2 * int64_t(cc - nrhs) * vstride;
    base[2 * int64_t(r) + (n & 1)] += v;
  }
};
// Far-field partial sums of K split s: complex column c = 6 rhs + component
// (V_D x, y, z, V_N x, y, z) at part[((rhs nseg + s) 12 + 2 comp + part) nobs + o].
struct FarOut {
  double* part;
  int nobs, nseg;
  __device__ __forceinline__ void put(int o, int n, int s, double v) const {
    const int cc = n >> 1, r = cc / 6, comp = cc - 6 * r;
    part[((int64_t(r) * nseg + s) * 12 + 2 * comp + (n & 1)) * nobs + o] = v;
  }
};
// Antipodal-pair partial sums of K split s: tile row r -> direction
// 64 (r / 128) + r % 64, trig = (r % 128) / 64 (cos, sin); real column n ->
// rhs, component and part (Re, Im J) at
// part[((rhs nseg + s) 24 + 4 comp + 2 trig + part) nh + o].
struct FarPairOut {
  double* part;
  int nh, nseg;
  __device__ __forceinline__ void put(int r, int n, int s, double v) const {
    const int rl = r & 127, o = ((r >> 7) << 6) + (rl & 63);
    if (o >= nh) return;
    const int cc = n >> 1, rr = cc / 6, comp = cc - 6 * rr;
    part[((int64_t(rr) * nseg + s) * 24 + 4 * comp + 2 * (rl >> 6) + (n & 1)) * nh + o] = v;
  }
};

// out(rows x Nr) = sum over K of Ahat Bhat; blockIdx.z picks the pair
// (s0, o0) for z = 0, else (s1, o1): two products in one launch, or (with
// s0 = s1) the K splits of the far field, whose source reads blockIdx.z.
template <typename Src, typename Out>
__global__ __launch_bounds__(256, 2) void k_mfma64(Src s0, Out o0, Src s1, Out o1, int rows, int Nr) {
  __shared__ double As[2][M64_BK * M64_LD];
  __shared__ double Bs[2][M64_BK * M64_LD];
  const int z = blockIdx.z;
  const Src src = z == 0 ? s0 : s1;  // by value: selected in scalar registers
  const Out out = z == 0 ? o0 : o1;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = blockIdx.y * M64_BM, n0 = blockIdx.x * M64_BN;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
  const int li = lane & 15, lk = lane >> 4;
  md4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = md4{0.0, 0.0, 0.0, 0.0};
  const int nt = src.ntiles();
  double ra[8], rb[8];
  const int srow = t >> 1, sk = 8 * (t & 1);
  auto sstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if constexpr (Src::A_PAIRS)  // row t / 4 (cos) and 64 + t / 4 (sin), K column 4 (t % 4) + q / 2
        As[buf][(4 * (t & 3) + (q >> 1)) * M64_LD + (q & 1) * 64 + (t >> 2)] = ra[q];
      else
        As[buf][(sk + q) * M64_LD + srow] = ra[q];
      Bs[buf][(sk + q) * M64_LD + srow] = rb[q];
    }
  };
  if (nt > 0) {
    src.load(0, m0, n0, rows, Nr, t, ra, rb);
    sstore(0);
  }
  __syncthreads();
  for (int kt = 0; kt < nt; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nt) src.load(kt + 1, m0, n0, rows, Nr, t, ra, rb);
#pragma unroll
    for (int kk = 0; kk < M64_BK / 4; ++kk) {
      const double* pa = &As[buf][(4 * kk + lk) * M64_LD + wr + li];
      const double* pb = &Bs[buf][(4 * kk + lk) * M64_LD + wc + li];
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = pa[16 * i];
        b[i] = pb[16 * i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nt) sstore(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + wc + 16 * j + li;
      if (n >= Nr) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = m0 + wr + 16 * i + lk + 4 * v;
        if (r < rows) out.put(r, n, z, acc[i][j][v]);
      }
    }
}

// Bhat^T of the PMCHWT right-hand block of one medium (k scaling inside), as
// the FP32 k_mfma_rhs: B1 for C ([X_D | X_N]), B2 for S ([X_N / k | -k X_D]).
__global__ void k_mfma64_rhs(const double* __restrict__ xD, const double* __restrict__ xN, int64_t vstride, int E,
                             int Kt, int nrhs, double kr, double ki, double* __restrict__ B1,
                             double* __restrict__ B2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (2 * k >= Kt) return;
  double b1r = 0, b1i = 0, b2r = 0, b2i = 0;
  if (k < E) {
    const double k2 = kr * kr + ki * ki;
    const double ikr = kr / k2, iki = -ki / k2;
    if (c < nrhs) {
      const double* d = xD + 2 * (int64_t(c) * vstride + k);
      const double* n = xN + 2 * (int64_t(c) * vstride + k);
      b1r = d[0];
      b1i = d[1];
      b2r = n[0] * ikr - n[1] * iki;
      b2i = n[0] * iki + n[1] * ikr;
    } else {
      const double* d = xD + 2 * (int64_t(c - nrhs) * vstride + k);
      const double* n = xN + 2 * (int64_t(c - nrhs) * vstride + k);
      b1r = n[0];
      b1i = n[1];
      b2r = -(kr * d[0] - ki * d[1]);
      b2i = -(kr * d[1] + ki * d[0]);
    }
  }
  const int64_t r0 = int64_t(2 * c) * Kt + 2 * k, r1 = r0 + Kt;
  B1[r0] = b1r;
  B1[r0 + 1] = -b1i;
  B1[r1] = b1i;
  B1[r1 + 1] = b1r;
  B2[r0] = b2r;
  B2[r0 + 1] = -b2i;
  B2[r1] = b2i;
  B2[r1 + 1] = b2r;
}

void launch_mfma64_comb(const double* C, const double* S1, const double* S2, int64_t ld, int rows, int cols,
                        const double* xD, const double* xN, double* yD, double* yN, int nrhs, int64_t vstride,
                        double* BD, double* BN, hipStream_t st) {
  const int Kt = int(2 * ld);  // ld a multiple of 8: Kt a multiple of 16
  const int Nr = 2 * nrhs;
  const dim3 gb(unsigned((Kt / 2 + 255) / 256), unsigned(nrhs));
  hipLaunchKernelGGL(k_mfma_rhs_plain<double>, gb, dim3(256), 0, st, xD, vstride, cols, Kt, BD);
  hipLaunchKernelGGL(k_mfma_rhs_plain<double>, gb, dim3(256), 0, st, xN, vstride, cols, Kt, BN);
  const Mem2Src sd{C, BD, Kt, 2 * ld, S1, BN, Kt, 2 * ld}, sn{C, BN, Kt, 2 * ld, S2, BD, Kt, 2 * ld};
  const dim3 grid(unsigned((Nr + M64_BN - 1) / M64_BN), unsigned((rows + M64_BM - 1) / M64_BM), 2);
  hipLaunchKernelGGL((k_mfma64<Mem2Src, Cplx64Out>), grid, dim3(256), 0, st, sd, Cplx64Out{yD, vstride}, sn,
                     Cplx64Out{yN, vstride}, rows, Nr);
}

void launch_mfma64_pmchwt(const double* S, const double* C, int64_t ld, int rows, int cols, double kr, double ki,
                          const double* xD, const double* xN, double* yD, double* yN, int nrhs, int64_t vstride,
                          double* B1, double* B2, hipStream_t st) {
  const int Kt = int(2 * ld);
  const int Nr = 4 * nrhs;
  hipLaunchKernelGGL(k_mfma64_rhs, dim3(unsigned((Kt / 2 + 255) / 256), unsigned(2 * nrhs)), dim3(256), 0, st, xD, xN,
                     vstride, cols, Kt, nrhs, kr, ki, B1, B2);
  const Mem2Src src{C, B1, Kt, 2 * ld, S, B2, Kt, 2 * ld};
  const Pmchwt64Out out{yD, yN, vstride, nrhs};
  const dim3 grid(unsigned((Nr + M64_BN - 1) / M64_BN), unsigned((rows + M64_BM - 1) / M64_BM), 1);
  hipLaunchKernelGGL((k_mfma64<Mem2Src, Pmchwt64Out>), grid, dim3(256), 0, st, src, out, src, out, rows, Nr);
}

// ---------------------------------------------------------------------------
// Far field as a matrix product: V[o][c] = sum_p exp(-i k xh_o . y_p) J_c(y_p)
// for the 6 nrhs complex columns c = (rhs, component) of the weighted
// currents at the rule points (k_far_points), K split over blockIdx.z, then
// k_far_finish as for the VALU sum.
// ---------------------------------------------------------------------------

// Bhat^T[n][k] from J[rhs][p][12]: n = 2 (6 rhs + comp) + {0, 1}, k = 2 p + {0, 1}
// (zero for p >= npts up to Kt / 2)
__global__ void k_far_bhat(const double* __restrict__ J, int64_t npts, int Kt, int nrhs, double* __restrict__ B) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int cc = blockIdx.y;  // complex column 6 rhs + comp
  if (2 * p >= Kt) return;
  const int r = cc / 6, comp = cc - 6 * r;
  double br = 0.0, bi = 0.0;
  if (p < npts) {
    const double* j = J + 12 * (int64_t(r) * npts + p) + 2 * comp;
    br = j[0];
    bi = j[1];
  }
  const int64_t r0 = int64_t(2 * cc) * Kt + 2 * p, r1 = r0 + Kt;
  B[r0] = br;
  B[r0 + 1] = -bi;
  B[r1] = bi;
  B[r1 + 1] = br;
}

// K splits of a far-field product: the first count (at least 32 K tiles per
// split) whose workgroups fill the whole rounds of the chip's 512 slots (two
// workgroups per CU) to at least 85 %, else the one that fills them best
int far_nsplit(int64_t tiles, int nkt) {
  constexpr int64_t slots = 512;
  const int64_t cap = std::max<int64_t>(1, nkt / 32);
  int64_t best = 1;
  double best_eff = 0.0;
  for (int64_t ns = 1; ns <= cap; ++ns) {
    const int64_t w = tiles * ns, rounds = (w + slots - 1) / slots;
    const double eff = double(w) / double(rounds * slots);
    if (eff > best_eff) {
      best_eff = eff;
      best = ns;
    }
    if (eff >= 0.85) break;
  }
  return int(best);
}

FarMfmaPlan far_mfma_plan(int F, int nrhs, int nobs) {
  FarMfmaPlan p;
  p.npts = int64_t(F) * 6;
  p.Kt = int((2 * p.npts + M64_BK - 1) / M64_BK * M64_BK);
  p.Nr = 12 * nrhs;
  const int64_t tiles = int64_t((p.Nr + M64_BN - 1) / M64_BN) * ((nobs + M64_BM - 1) / M64_BM);
  const int nkt = p.Kt / M64_BK;
  p.nsplit = far_nsplit(tiles, nkt);
  p.rows = nobs;
  p.n_B = int64_t(p.Nr) * p.Kt;
  p.n_part = int64_t(nrhs) * p.nsplit * 12 * nobs;
  return p;
}

void launch_far_field_mfma(const AsmParams<double>& geo, const double* x, int64_t E_tot, int nrhs, double k,
                           const double* obs, int nobs, double* F_out, const FarMfmaPlan& plan, double* ypts,
                           double* J, double* B, double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_far_points, dim3(unsigned((plan.npts + 255) / 256)), dim3(256), 0, st, geo, x, E_tot, nrhs,
                     plan.npts, ypts, J);
  hipLaunchKernelGGL(k_far_bhat, dim3(unsigned((plan.Kt / 2 + 255) / 256), unsigned(6 * nrhs)), dim3(256), 0, st, J,
                     plan.npts, plan.Kt, nrhs, B);
  const int nkt = plan.Kt / M64_BK;
  const dim3 grid(unsigned((plan.Nr + M64_BN - 1) / M64_BN), unsigned((nobs + M64_BM - 1) / M64_BM),
                  unsigned(plan.nsplit));
  const FarSrc src{obs, ypts, B, plan.npts, plan.Kt, nobs, k, nkt, plan.nsplit};
  const FarOut out{part, nobs, plan.nsplit};
  hipLaunchKernelGGL((k_mfma64<FarSrc, FarOut>), grid, dim3(256), 0, st, src, out, src, out, nobs, plan.Nr);
  const int64_t n = int64_t(nobs) * nrhs;
  hipLaunchKernelGGL(k_far_finish, dim3(unsigned((n + 127) / 128)), dim3(128), 0, st, part, plan.nsplit, k, obs, nobs,
                     nrhs, F_out);
}

// ---------------------------------------------------------------------------
// Far field at nh directions and their antipodes: one FP64 GEMM of the
// cosine and sine rows (2 per direction) against the real and imaginary
// parts of the weighted currents, K = rule points, then k_far_finish_pair.
// ---------------------------------------------------------------------------

// B[12 r + c][p] = J[r][p][c] (c = 2 comp + {Re, Im}), zero for
// npts <= p < Kt: per rhs a transpose of the npts x 12 current table, 64
// points per workgroup through LDS (both sides coalesced)
__global__ __launch_bounds__(256) void k_far_bsplit(const double* __restrict__ J, int64_t npts, int Kt,
                                                    double* __restrict__ B) {
  __shared__ double s[64 * 13];  // point q at 13 q (padded row)
  const int64_t p0 = int64_t(blockIdx.x) * 64;
  const int r = blockIdx.y;
  const double* Jr = J + 12 * (int64_t(r) * npts + p0);
  for (int i = threadIdx.x; i < 64 * 12; i += 256) s[13 * (i / 12) + i % 12] = p0 + i / 12 < npts ? Jr[i] : 0.0;
  __syncthreads();
  for (int i = threadIdx.x; i < 64 * 12; i += 256) {
    const int c = i >> 6, q = i & 63;
    if (p0 + q < Kt) B[(12 * int64_t(r) + c) * Kt + p0 + q] = s[13 * q + c];
  }
}

FarMfmaPlan far_pair_plan(int F, int nrhs, int nh) {
  FarMfmaPlan p;
  p.npts = int64_t(F) * 6;
  p.Kt = int((p.npts + M64_BK - 1) / M64_BK * M64_BK);
  p.Nr = 12 * nrhs;
  p.rows = M64_BM * ((nh + M64_BM / 2 - 1) / (M64_BM / 2));
  const int64_t tiles = int64_t((p.Nr + M64_BN - 1) / M64_BN) * (p.rows / M64_BM);
  const int nkt = p.Kt / M64_BK;
  p.nsplit = far_nsplit(tiles, nkt);
  p.n_B = int64_t(p.Nr) * p.Kt;
  p.n_part = int64_t(nrhs) * p.nsplit * 24 * nh;
  return p;
}

void launch_far_field_pair(const AsmParams<double>& geo, const double* x, int64_t E_tot, int nrhs, double k,
                           const double* obs, int nh, double* F_out, const FarMfmaPlan& plan, double* ypts, double* J,
                           double* B, double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_far_points, dim3(unsigned((plan.npts + 255) / 256)), dim3(256), 0, st, geo, x, E_tot, nrhs,
                     plan.npts, ypts, J);
  hipLaunchKernelGGL(k_far_bsplit, dim3(unsigned((plan.Kt + 63) / 64), unsigned(nrhs)), dim3(256), 0, st, J,
                     plan.npts, plan.Kt, B);
  const int nkt = plan.Kt / M64_BK;
  const dim3 grid(unsigned((plan.Nr + M64_BN - 1) / M64_BN), unsigned(plan.rows / M64_BM), unsigned(plan.nsplit));
  const FarPairSrc src{obs, ypts, B, plan.npts, plan.Kt, nh, k, nkt, plan.nsplit};
  const FarPairOut out{part, nh, plan.nsplit};
  hipLaunchKernelGGL((k_mfma64<FarPairSrc, FarPairOut>), grid, dim3(256), 0, st, src, out, src, out, plan.rows,
                     plan.Nr);
  const int64_t n = int64_t(nh) * nrhs;
  hipLaunchKernelGGL(k_far_finish_pair, dim3(unsigned((n + 127) / 128)), dim3(128), 0, st, part, plan.nsplit, k, obs,
                     nh, nrhs, F_out);
}

}  // namespace pmchwt
