// Operator application and Krylov kernels (Section 3.2 product operator,
// GMRES of Section 4).
//
// Dense operators are HBM-bound at a few right-hand sides: each wavefront
// streams rows of S and C once for all vectors of the batch and accumulates in
// FP64 (also for FP32 storage).  Krylov vectors are complex128.
#include "common.hpp"
#include "kernels.hpp"

namespace pmchwt {

template <typename T>
__device__ __forceinline__ T wsum(T v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

template <typename M>
struct Pair2 {
  M re, im;
};

// ---------------------------------------------------------------------------
// yD += C xD + S (xN / k) ; yN += C xN + S (-k xD).  The two scaled vectors
// are formed per column in registers, so each row needs only two complex
// accumulators.  One wavefront streams ROWS rows (every x load from L2
// serves all of them); each lane loads two consecutive complex entries of S
// and C per step with one vector load (rows start on aligned boundaries: the
// leading dimension is a multiple of 4), marked non-temporal since the
// operator is read once per application.  FP64 accumulation for either
// storage type.
// ---------------------------------------------------------------------------
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));
template <typename M>
struct CPair {};
template <>
struct CPair<float> {
  typedef f4v T;
};
template <>
struct CPair<double> {
  typedef d4v T;
};

// rows per wavefront for NR right-hand sides (register budget)
template <typename M, int NR>
struct GemvRows {
  static constexpr int value = (sizeof(M) == 4 ? 8 : 4) / NR > 0 ? (sizeof(M) == 4 ? 8 : 4) / NR : 1;
};

// Rows of workgroup `blk` (four wavefronts of ROWS rows each).
template <typename M, int NR>
__device__ __forceinline__ void gemv_pmchwt_rows(const M* __restrict__ S, const M* __restrict__ C, int64_t ld,
                                                 int rows, int cols, double kr, double ki,
                                                 const double* __restrict__ xD, const double* __restrict__ xN,
                                                 double* yD, double* yN, int64_t vstride, int blk) {
  constexpr int ROWS = GemvRows<M, NR>::value;
  typedef typename CPair<M>::T V;
  const int lane = threadIdx.x & 63;
  const int row0 = ROWS * (blk * (blockDim.x / 64) + threadIdx.x / 64);
  if (row0 >= rows) return;
  const V* Sv[ROWS];
  const V* Cv[ROWS];
#pragma unroll
  for (int h = 0; h < ROWS; ++h) {
    const int r = min(row0 + h, rows - 1);
    Sv[h] = reinterpret_cast<const V*>(S + 2 * int64_t(r) * ld);
    Cv[h] = reinterpret_cast<const V*>(C + 2 * int64_t(r) * ld);
  }
  const double k2 = kr * kr + ki * ki;
  const double ikr = kr / k2, iki = -ki / k2;  // 1/k
  double a[ROWS][NR][4];
#pragma unroll
  for (int h = 0; h < ROWS; ++h)
#pragma unroll
    for (int r = 0; r < NR; ++r) a[h][r][0] = a[h][r][1] = a[h][r][2] = a[h][r][3] = 0.0;
  const int np = (cols + 1) >> 1;
  for (int q = lane; q < np; q += 64) {
    V sv[ROWS], cv[ROWS];
#pragma unroll
    for (int h = 0; h < ROWS; ++h) {
      sv[h] = __builtin_nontemporal_load(&Sv[h][q]);
      cv[h] = __builtin_nontemporal_load(&Cv[h][q]);
    }
    const int j = 2 * q;
    const bool pair = j + 1 < cols;
    // xd, xn and the scaled p = xN / k, m = -k xD; two columns each
    double xd[NR][4], xn[NR][4], pv[NR][4], mv[NR][4];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double2* pd = reinterpret_cast<const double2*>(xD + 2 * (int64_t(r) * vstride + j));
      const double2* pn = reinterpret_cast<const double2*>(xN + 2 * (int64_t(r) * vstride + j));
      const double2 d0 = pd[0], n0 = pn[0];
      const double2 d1 = pair ? pd[1] : double2{0.0, 0.0};
      const double2 n1 = pair ? pn[1] : double2{0.0, 0.0};
      xd[r][0] = d0.x;
      xd[r][1] = d0.y;
      xd[r][2] = d1.x;
      xd[r][3] = d1.y;
      xn[r][0] = n0.x;
      xn[r][1] = n0.y;
      xn[r][2] = n1.x;
      xn[r][3] = n1.y;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        pv[r][2 * u] = xn[r][2 * u] * ikr - xn[r][2 * u + 1] * iki;
        pv[r][2 * u + 1] = xn[r][2 * u] * iki + xn[r][2 * u + 1] * ikr;
        mv[r][2 * u] = -(kr * xd[r][2 * u] - ki * xd[r][2 * u + 1]);
        mv[r][2 * u + 1] = -(kr * xd[r][2 * u + 1] + ki * xd[r][2 * u]);
      }
    }
#pragma unroll
    for (int h = 0; h < ROWS; ++h) {
      const double s4[4] = {double(sv[h].x), double(sv[h].y), double(sv[h].z), double(sv[h].w)};
      const double c4[4] = {double(cv[h].x), double(cv[h].y), double(cv[h].z), double(cv[h].w)};
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const double sr = s4[2 * u], si = s4[2 * u + 1], cr = c4[2 * u], ci = c4[2 * u + 1];
          a[h][r][0] += cr * xd[r][2 * u] - ci * xd[r][2 * u + 1] + sr * pv[r][2 * u] - si * pv[r][2 * u + 1];
          a[h][r][1] += cr * xd[r][2 * u + 1] + ci * xd[r][2 * u] + sr * pv[r][2 * u + 1] + si * pv[r][2 * u];
          a[h][r][2] += cr * xn[r][2 * u] - ci * xn[r][2 * u + 1] + sr * mv[r][2 * u] - si * mv[r][2 * u + 1];
          a[h][r][3] += cr * xn[r][2 * u + 1] + ci * xn[r][2 * u] + sr * mv[r][2 * u + 1] + si * mv[r][2 * u];
        }
    }
  }
#pragma unroll
  for (int h = 0; h < ROWS; ++h)
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) a[h][r][q] = wsum(a[h][r][q]);
  if (lane == 0) {
#pragma unroll
    for (int h = 0; h < ROWS; ++h) {
      if (row0 + h >= rows) break;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        double* yd = yD + 2 * (int64_t(r) * vstride + row0 + h);
        double* yn = yN + 2 * (int64_t(r) * vstride + row0 + h);
        yd[0] += a[h][r][0];
        yd[1] += a[h][r][1];
        yn[0] += a[h][r][2];
        yn[1] += a[h][r][3];
      }
    }
  }
}

template <typename M, int NR>
__global__ __launch_bounds__(256) void k_gemv_pmchwt(const M* __restrict__ S, const M* __restrict__ C,
                                                     int64_t ld, int rows, int cols, double kr, double ki,
                                                     const double* __restrict__ xD,
                                                     const double* __restrict__ xN, double* yD, double* yN,
                                                     int64_t vstride) {
  gemv_pmchwt_rows<M, NR>(S, C, ld, rows, cols, kr, ki, xD, xN, yD, yN, vstride, blockIdx.x);
}

// Several independent products in one launch (the operators of different
// problems): workgroup b belongs to the job with block0 <= b < next block0
// and runs exactly the rows a launch of that job alone would give it.
template <typename M, int NR>
__global__ __launch_bounds__(256) void k_gemv_pmchwt_grouped(const GemvJob<M>* __restrict__ jobs, int njobs) {
  int lo = 0, hi = njobs - 1;
  const int b = blockIdx.x;
  while (lo < hi) {  // last job with block0 <= b
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].block0 <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  const GemvJob<M> j = jobs[lo];
  gemv_pmchwt_rows<M, NR>(j.S, j.C, j.ld, j.rows, j.cols, j.kr, j.ki, j.xD, j.xN, j.yD, j.yN, j.vstride,
                          b - j.block0);
}

template <typename M>
int gemv_blocks(int rows, int nr) {
  const int rpw = nr >= 4 ? GemvRows<M, 4>::value : (nr >= 2 ? GemvRows<M, 2>::value : GemvRows<M, 1>::value);
  return (rows + 4 * rpw - 1) / (4 * rpw);
}

template <typename M>
void launch_gemv_pmchwt_grouped(const GemvJob<M>* jobs_dev, int njobs, int nr, int total_blocks, hipStream_t st) {
  if (njobs == 0) return;
  const dim3 grid{static_cast<unsigned>(total_blocks)}, block{256};
  if (nr == 4)
    hipLaunchKernelGGL((k_gemv_pmchwt_grouped<M, 4>), grid, block, 0, st, jobs_dev, njobs);
  else if (nr == 2)
    hipLaunchKernelGGL((k_gemv_pmchwt_grouped<M, 2>), grid, block, 0, st, jobs_dev, njobs);
  else
    hipLaunchKernelGGL((k_gemv_pmchwt_grouped<M, 1>), grid, block, 0, st, jobs_dev, njobs);
}
template void launch_gemv_pmchwt_grouped<float>(const GemvJob<float>*, int, int, int, hipStream_t);
template void launch_gemv_pmchwt_grouped<double>(const GemvJob<double>*, int, int, int, hipStream_t);
template int gemv_blocks<float>(int, int);
template int gemv_blocks<double>(int, int);

// Single scatterer: A = A^e + A^i applied from three pre-combined matrices
//   C = C^e + C^i,  S1 = S^e/k_e + S^i/k_i,  S2 = -(k_e S^e + k_i S^i),
//   yD (+)= C xD + S1 xN,  yN (+)= C xN + S2 xD
// (three operator reads per row instead of four).  A workgroup has four
// wavefronts; KS of them share a group of ROWS rows and take consecutive
// column ranges (more wavefronts in flight when the rows alone give too few),
// their partial sums added in a fixed order through LDS.
template <typename M, int NR, int KS>
__global__ __launch_bounds__(256) void k_gemv_pmchwt3(const M* __restrict__ C, const M* __restrict__ S1,
                                                      const M* __restrict__ S2, int64_t ld, int rows, int cols,
                                                      const double* __restrict__ xD, const double* __restrict__ xN,
                                                      double* yD, double* yN, int64_t vstride, int acc) {
  constexpr int ROWS = GemvRows<M, NR>::value;
  typedef typename CPair<M>::T V;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int part = wv % KS;
  const int row0 = ROWS * (blockIdx.x * (4 / KS) + wv / KS);
  const bool live = row0 < rows;  // no early exit: every wavefront reaches the barrier
  const V* Cv[ROWS];
  const V* Av[ROWS];
  const V* Bv[ROWS];
#pragma unroll
  for (int h = 0; h < ROWS; ++h) {
    const int r = min(row0 + h, rows - 1);
    Cv[h] = reinterpret_cast<const V*>(C + 2 * int64_t(r) * ld);
    Av[h] = reinterpret_cast<const V*>(S1 + 2 * int64_t(r) * ld);
    Bv[h] = reinterpret_cast<const V*>(S2 + 2 * int64_t(r) * ld);
  }
  double a[ROWS][NR][4];
#pragma unroll
  for (int h = 0; h < ROWS; ++h)
#pragma unroll
    for (int r = 0; r < NR; ++r) a[h][r][0] = a[h][r][1] = a[h][r][2] = a[h][r][3] = 0.0;
  const int np = (cols + 1) >> 1;
  const int q0 = int(int64_t(np) * part / KS), q1 = live ? int(int64_t(np) * (part + 1) / KS) : q0;
  for (int q = q0 + lane; q < q1; q += 64) {
    V cv[ROWS], av[ROWS], bv[ROWS];
#pragma unroll
    for (int h = 0; h < ROWS; ++h) {
      cv[h] = __builtin_nontemporal_load(&Cv[h][q]);
      av[h] = __builtin_nontemporal_load(&Av[h][q]);
      bv[h] = __builtin_nontemporal_load(&Bv[h][q]);
    }
    const int j = 2 * q;
    const bool pair = j + 1 < cols;
    double xd[NR][4], xn[NR][4];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double2* pd = reinterpret_cast<const double2*>(xD + 2 * (int64_t(r) * vstride + j));
      const double2* pn = reinterpret_cast<const double2*>(xN + 2 * (int64_t(r) * vstride + j));
      const double2 d0 = pd[0], n0 = pn[0];
      const double2 d1 = pair ? pd[1] : double2{0.0, 0.0};
      const double2 n1 = pair ? pn[1] : double2{0.0, 0.0};
      xd[r][0] = d0.x;
      xd[r][1] = d0.y;
      xd[r][2] = d1.x;
      xd[r][3] = d1.y;
      xn[r][0] = n0.x;
      xn[r][1] = n0.y;
      xn[r][2] = n1.x;
      xn[r][3] = n1.y;
    }
#pragma unroll
    for (int h = 0; h < ROWS; ++h) {
      const double c4[4] = {double(cv[h].x), double(cv[h].y), double(cv[h].z), double(cv[h].w)};
      const double s4[4] = {double(av[h].x), double(av[h].y), double(av[h].z), double(av[h].w)};
      const double t4[4] = {double(bv[h].x), double(bv[h].y), double(bv[h].z), double(bv[h].w)};
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const double cr = c4[2 * u], ci = c4[2 * u + 1], sr = s4[2 * u], si = s4[2 * u + 1];
          const double tr = t4[2 * u], ti = t4[2 * u + 1];
          const double dr = xd[r][2 * u], di = xd[r][2 * u + 1], nr = xn[r][2 * u], ni = xn[r][2 * u + 1];
          a[h][r][0] += cr * dr - ci * di + sr * nr - si * ni;
          a[h][r][1] += cr * di + ci * dr + sr * ni + si * nr;
          a[h][r][2] += cr * nr - ci * ni + tr * dr - ti * di;
          a[h][r][3] += cr * ni + ci * nr + tr * di + ti * dr;
        }
    }
  }
#pragma unroll
  for (int h = 0; h < ROWS; ++h)
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) a[h][r][q] = wsum(a[h][r][q]);
  if (KS > 1) {
    __shared__ double red[4][ROWS * NR * 4];
    if (lane == 0 && part > 0) {
#pragma unroll
      for (int h = 0; h < ROWS; ++h)
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
          for (int q = 0; q < 4; ++q) red[wv][(h * NR + r) * 4 + q] = a[h][r][q];
    }
    __syncthreads();
    if (lane == 0 && part == 0) {
#pragma unroll
      for (int p = 1; p < KS; ++p)
#pragma unroll
        for (int h = 0; h < ROWS; ++h)
#pragma unroll
          for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int q = 0; q < 4; ++q) a[h][r][q] += red[wv + p][(h * NR + r) * 4 + q];
    }
  }
  if (lane == 0 && part == 0 && live) {
#pragma unroll
    for (int h = 0; h < ROWS; ++h) {
      if (row0 + h >= rows) break;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        double* yd = yD + 2 * (int64_t(r) * vstride + row0 + h);
        double* yn = yN + 2 * (int64_t(r) * vstride + row0 + h);
        const double o0 = acc ? yd[0] : 0.0, o1 = acc ? yd[1] : 0.0, o2 = acc ? yn[0] : 0.0, o3 = acc ? yn[1] : 0.0;
        yd[0] = o0 + a[h][r][0];
        yd[1] = o1 + a[h][r][1];
        yn[0] = o2 + a[h][r][2];
        yn[1] = o3 + a[h][r][3];
      }
    }
  }
}

template <typename M, int NR>
static void gemv3_launch(int rows, const M* C, const M* S1, const M* S2, int64_t ld, int cols, const double* xd,
                         const double* xn, double* yd, double* yn, int64_t vstride, bool acc, hipStream_t st) {
  constexpr int ROWS = GemvRows<M, NR>::value;
  const int groups = (rows + ROWS - 1) / ROWS;
  // split the columns of a row group over 4 or 2 wavefronts while the row
  // groups alone are fewer than one per CU / one per SIMD (measured on the
  // 7680-column operator: 2-way equal to 1-way; on 1920 and 3840 columns:
  // 2.0x and 1.45x faster than 1-way)
  if (groups <= 256)
    hipLaunchKernelGGL((k_gemv_pmchwt3<M, NR, 4>), dim3(unsigned(groups)), dim3(256), 0, st, C, S1, S2, ld, rows, cols,
                       xd, xn, yd, yn, vstride, int(acc));
  else if (groups <= 1024)
    hipLaunchKernelGGL((k_gemv_pmchwt3<M, NR, 2>), dim3(unsigned((groups + 1) / 2)), dim3(256), 0, st, C, S1, S2, ld,
                       rows, cols, xd, xn, yd, yn, vstride, int(acc));
  else
    hipLaunchKernelGGL((k_gemv_pmchwt3<M, NR, 1>), dim3(unsigned((groups + 3) / 4)), dim3(256), 0, st, C, S1, S2, ld,
                       rows, cols, xd, xn, yd, yn, vstride, int(acc));
}

template <typename M>
void launch_gemv_pmchwt3(const M* C, const M* S1, const M* S2, int64_t ld, int rows, int cols, const double* xD,
                         const double* xN, double* yD, double* yN, int nrhs, int64_t vstride, hipStream_t st,
                         bool acc) {
  for (int r0 = 0; r0 < nrhs;) {
    const int left = nrhs - r0;
    const double* xd = xD + 2 * int64_t(r0) * vstride;
    const double* xn = xN + 2 * int64_t(r0) * vstride;
    double* yd = yD + 2 * int64_t(r0) * vstride;
    double* yn = yN + 2 * int64_t(r0) * vstride;
    if (left >= 4) {
      gemv3_launch<M, 4>(rows, C, S1, S2, ld, cols, xd, xn, yd, yn, vstride, acc, st);
      r0 += 4;
    } else if (left >= 2) {
      gemv3_launch<M, 2>(rows, C, S1, S2, ld, cols, xd, xn, yd, yn, vstride, acc, st);
      r0 += 2;
    } else {
      gemv3_launch<M, 1>(rows, C, S1, S2, ld, cols, xd, xn, yd, yn, vstride, acc, st);
      r0 += 1;
    }
  }
}
template void launch_gemv_pmchwt3<float>(const float*, const float*, const float*, int64_t, int, int, const double*,
                                         const double*, double*, double*, int, int64_t, hipStream_t, bool);
template void launch_gemv_pmchwt3<double>(const double*, const double*, const double*, int64_t, int, int,
                                          const double*, const double*, double*, double*, int, int64_t, hipStream_t,
                                          bool);

// C = Ce + Ci, S1 = Se/ke + Si/ki, S2 = -(ke Se + ki Si) of complex entry q
// (out: C, S1, S2 as re/im pairs, rounded to the storage type)
template <typename M>
__device__ __forceinline__ void combine_entry(const M* Se, const M* Ce, const M* Si, const M* Ci, int64_t q,
                                              double ke, double kir, double kii, M out[6]) {
  const double ser = Se[2 * q], sei = Se[2 * q + 1], sir = Si[2 * q], sii = Si[2 * q + 1];
  out[0] = M(double(Ce[2 * q]) + double(Ci[2 * q]));
  out[1] = M(double(Ce[2 * q + 1]) + double(Ci[2 * q + 1]));
  const double k2 = kir * kir + kii * kii, ir = kir / k2, ii = -kii / k2;  // 1/ki
  out[2] = M(ser / ke + (sir * ir - sii * ii));
  out[3] = M(sei / ke + (sir * ii + sii * ir));
  out[4] = M(-(ke * ser + (kir * sir - kii * sii)));
  out[5] = M(-(ke * sei + (kir * sii + kii * sir)));
}

template <typename M>
__global__ void k_combine3(const M* Se, const M* Ce, const M* Si, const M* Ci, int64_t n, double ke, double kir,
                           double kii, M* C, M* S1, M* S2) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= n) return;
  M o[6];
  combine_entry(Se, Ce, Si, Ci, q, ke, kir, kii, o);
  C[2 * q] = o[0];
  C[2 * q + 1] = o[1];
  S1[2 * q] = o[2];
  S1[2 * q + 1] = o[3];
  S2[2 * q] = o[4];
  S2[2 * q + 1] = o[5];
}

template <typename M>
void launch_combine3(const M* Se, const M* Ce, const M* Si, const M* Ci, int64_t n, double ke, double kir, double kii,
                     M* C, M* S1, M* S2, hipStream_t st) {
  hipLaunchKernelGGL((k_combine3<M>), dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, Se, Ce, Si, Ci, n, ke, kir,
                     kii, C, S1, S2);
}
template void launch_combine3<float>(const float*, const float*, const float*, const float*, int64_t, double, double,
                                     double, float*, float*, float*, hipStream_t);
template void launch_combine3<double>(const double*, const double*, const double*, const double*, int64_t, double,
                                      double, double, double*, double*, double*, hipStream_t);

// ---------------------------------------------------------------------------
// Symmetric-tile product for one right-hand side.
//
// C, S1 and S2 are complex symmetric up to the quadrature of the singular
// pairs: S and C are symmetric bilinear forms on one space (test = trial,
// Section 3.1), every regular pair is integrated with the same rule from
// either side, and only the Sauter-Schwab rules of pairs sharing a vertex
// give X_rc != X_cr.  The operator is stored as its upper SYM_T x SYM_T tiles
// (I <= J; diagonal tiles whole), so one product reads half the bytes: tile
// (I, J) gives row sums for block row I and, transposed, column sums for block
// row J.  Entries below the diagonal tiles that singular pairs touch get the
// exact difference X_rc - X_cr from a CSR correction, so the product equals
// the one with the full matrices up to rounding.
//
// Tile t = (I, J) holds three T x T complex blocks (C, S1, S2) with their
// rows interleaved (row r of C, of S1, of S2, then row r + 1), so that one
// step of the product reads one contiguous span rather than three streams
// a block apart; entries outside the n x n operator are zero.  Partial sums: slot (K, s) of
// T rows x 4 doubles (yD re/im, yN re/im) is written by exactly one tile
// (row sums of (K, s) for K <= s, column sums of (s, K) for K > s) and added
// in slot order by k_sym_reduce.
// ---------------------------------------------------------------------------
template <typename M, int T>
__global__ void k_pack_sym3(const M* __restrict__ Se, const M* __restrict__ Ce, const M* __restrict__ Si,
                            const M* __restrict__ Ci, int64_t ld, int n, const int32_t* __restrict__ tij,
                            double ke, double kir, double kii, M* __restrict__ P) {
  constexpr int64_t MAT = int64_t(T) * T * 2;
  const int64_t q = int64_t(blockIdx.x) * 256 + threadIdx.x;  // T*T is a multiple of 256: no tail
  const int64_t t = q / (int64_t(T) * T);
  const int w = int(q - t * T * T), r = w / T, cc = w - r * T;
  const int R = tij[2 * t] * T + r, Cc = tij[2 * t + 1] * T + cc;
  M o[6] = {M(0), M(0), M(0), M(0), M(0), M(0)};
  if (R < n && Cc < n) combine_entry(Se, Ce, Si, Ci, int64_t(R) * ld + Cc, ke, kir, kii, o);
  // rows of the three blocks interleaved: tile t, row r, block b, column cc
  M* b = P + t * 3 * MAT + int64_t(r) * 6 * T + 2 * cc;
  b[0] = o[0];
  b[1] = o[1];
  b[2 * T] = o[2];
  b[2 * T + 1] = o[3];
  b[4 * T] = o[4];
  b[4 * T + 1] = o[5];
}

// correction entry k at (R, Cc), tile(R) > tile(Cc): X_RCc - X_CcR for the
// three combined matrices, both taken as stored (rounded to M)
template <typename M>
__global__ void k_sym_corr(const M* __restrict__ Se, const M* __restrict__ Ce, const M* __restrict__ Si,
                           const M* __restrict__ Ci, int64_t ld, const int32_t* __restrict__ crow,
                           const int32_t* __restrict__ col, int64_t nnz, double ke, double kir, double kii,
                           M* __restrict__ val) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  const int R = crow[k], Cc = col[k];
  M a[6], b[6];
  combine_entry(Se, Ce, Si, Ci, int64_t(R) * ld + Cc, ke, kir, kii, a);
  combine_entry(Se, Ce, Si, Ci, int64_t(Cc) * ld + R, ke, kir, kii, b);
#pragma unroll
  for (int q = 0; q < 6; ++q) val[6 * k + q] = M(double(a[q]) - double(b[q]));
}

// sum of the signed singular items of one correction entry, per operator
// (Se, Ce, Si, Ci): items (blk entry << 1 | negate), blk entries 4 complex
__device__ __forceinline__ void sing_item_sum(const int64_t* ptr, const int32_t* item, const double* blk, int64_t k,
                                              double out[8]) {
#pragma unroll
  for (int q = 0; q < 8; ++q) out[q] = 0.0;
  for (int64_t t = ptr[k]; t < ptr[k + 1]; ++t) {
    const int32_t it = item[t];
    const double sg = (it & 1) ? -1.0 : 1.0;
    const double* b = blk + 8 * int64_t(it >> 1);
#pragma unroll
    for (int q = 0; q < 8; ++q) out[q] += sg * b[q];
  }
}

template <typename M>
__global__ void k_sym_corr_sing(const int64_t* __restrict__ ptr, const int32_t* __restrict__ item,
                                const double* __restrict__ blk, int64_t nnz, double ke, double kir, double kii,
                                M* __restrict__ val) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  double d[8];
  sing_item_sum(ptr, item, blk, k, d);
  // the combination of combine_entry: C = Ce + Ci, S1 = Se/ke + Si/ki, S2 = -(ke Se + ki Si)
  const double ser = d[0], sei = d[1], cer = d[2], cei = d[3], sir = d[4], sii = d[5], cir = d[6], cii = d[7];
  const double k2 = kir * kir + kii * kii, ir = kir / k2, ii = -kii / k2;
  M* o = val + 6 * k;
  o[0] = M(cer + cir);
  o[1] = M(cei + cii);
  o[2] = M(ser / ke + (sir * ir - sii * ii));
  o[3] = M(sei / ke + (sir * ii + sii * ir));
  o[4] = M(-(ke * ser + (kir * sir - kii * sii)));
  o[5] = M(-(ke * sei + (kir * sii + kii * sir)));
}

template <typename M>
void launch_sym_corr_sing(const int64_t* ptr, const int32_t* item, const double* blk, int64_t nnz, double ke,
                          double kir, double kii, M* val, hipStream_t st) {
  if (nnz == 0) return;
  hipLaunchKernelGGL((k_sym_corr_sing<M>), dim3(unsigned((nnz + 255) / 256)), dim3(256), 0, st, ptr, item, blk, nnz,
                     ke, kir, kii, val);
}

// X[r][c] = X[c][r] for tile(r) > tile(c): 32 x 32 complex blocks through LDS
// (coalesced reads along the source rows, coalesced writes along the
// destination rows); blocks outside the strictly lower tiles exit
template <typename M>
__global__ __launch_bounds__(256) void k_mirror_lower(M* X, int64_t ld, int n) {
  __shared__ M sre[32][33], sim[32][33];
  const int R0 = blockIdx.y * 32, C0 = blockIdx.x * 32;
  if (R0 / SYM_T <= C0 / SYM_T) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 8 rows of 32 per pass
  for (int y = ty; y < 32; y += 8) {  // source rows C0 + y, columns R0 + tx
    const int sr = C0 + y, sc = R0 + tx;
    if (sr < n && sc < n) {
      sre[y][tx] = X[2 * (int64_t(sr) * ld + sc)];
      sim[y][tx] = X[2 * (int64_t(sr) * ld + sc) + 1];
    }
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {  // destination rows R0 + y, columns C0 + tx
    const int dr = R0 + y, dc = C0 + tx;
    if (dr < n && dc < n) {
      X[2 * (int64_t(dr) * ld + dc)] = sre[tx][y];
      X[2 * (int64_t(dr) * ld + dc) + 1] = sim[tx][y];
    }
  }
}

// correction entries after the mirror: X_rc += sing_rc - sing_cr of operator op
template <typename M>
__global__ void k_mirror_fix(M* X, int64_t ld, const int32_t* __restrict__ crow, const int32_t* __restrict__ col,
                             const int64_t* __restrict__ ptr, const int32_t* __restrict__ item,
                             const double* __restrict__ blk, int64_t nnz, int op) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  double d[8];
  sing_item_sum(ptr, item, blk, k, d);
  M* x = X + 2 * (int64_t(crow[k]) * ld + col[k]);
  x[0] = M(double(x[0]) + d[2 * op]);
  x[1] = M(double(x[1]) + d[2 * op + 1]);
}

template <typename M>
void launch_mirror_lower(M* X, int64_t ld, int n, const int32_t* crow, const int32_t* col, const int64_t* ptr,
                         const int32_t* item, const double* blk, int64_t nnz, int op, hipStream_t st) {
  const unsigned nb = unsigned((n + 31) / 32);
  hipLaunchKernelGGL((k_mirror_lower<M>), dim3(nb, nb), dim3(256), 0, st, X, ld, n);
  if (nnz > 0)
    hipLaunchKernelGGL((k_mirror_fix<M>), dim3(unsigned((nnz + 255) / 256)), dim3(256), 0, st, X, ld, crow, col, ptr,
                       item, blk, nnz, op);
}

// lane v of a 16-lane row moved by a DPP pattern (both 32-bit halves)
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int64_t b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp(int(uint32_t(b)), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(int(uint32_t(uint64_t(b) >> 32)), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(int64_t((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo)));
}

// sum over aligned groups of L lanes, every lane of a group gets it; within
// the rows of 16 lanes by DPP (swap neighbours, swap pairs, mirror halves of
// 8, mirror the row), across rows by shuffles
template <int L>
__device__ __forceinline__ double row_sum(double v) {
  if constexpr (L == 16 || L == 32) {
    v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_move<0x141>(v);  // row_half_mirror
    v += dpp_move<0x140>(v);  // row_mirror
    if constexpr (L == 32) v += __shfl_xor(v, 16, WAVE);
  } else {
#pragma unroll
    for (int o = L / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, WAVE);
  }
  return v;
}

// One workgroup per tile.  Wavefront w takes rows [w T/4, (w+1) T/4), G RPS
// at a time (G = 64 / LPR row groups of LPR lanes): row group g = lane / LPR
// reads rows g, g + G, ..., lane cl = lane % LPR holding columns
// 2(cl + LPR k) + {0, 1}, k < T / (2 LPR), of all three blocks (contiguous
// LPR-lane segments per load).  Row sums: FP64 per lane, then over the LPR
// lanes.  Column sums: per lane over its rows, then over the G row groups
// (shuffles) and the four wavefronts (LDS), in that fixed order.  XREG keeps
// the lane's column x values in registers (else they are re-read from LDS
// every step); WPE is a minimum of wavefronts per SIMD for the register
// allocator.
template <typename M, int T, int LPR, int RPS, int WPE = 1, bool XREG = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void k_gemv_sym3(const M* __restrict__ P, const int32_t* __restrict__ tij, int nt,
                                                   int n, const double* __restrict__ xD,
                                                   const double* __restrict__ xN, double* __restrict__ part) {
  typedef typename CPair<M>::T V;  // two complex entries
  constexpr int G = 64 / LPR;      // row groups per wavefront
  constexpr int NU = T / (2 * LPR);  // vector loads per lane, row and block
  constexpr int RW = T / 4;        // rows per wavefront
  constexpr int64_t MATV = int64_t(T) * T / 2;
  static_assert(NU >= 1 && RW % (G * RPS) == 0, "tile, lanes per row and rows per step do not fit");
  const int t = blockIdx.x;
  const int I = tij[2 * t], J = tij[2 * t + 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane / LPR, cl = lane % LPR;
  __shared__ double xr[T][4];  // x of the tile's rows (block row I)
  __shared__ double xk[T][4];  // x of the tile's columns (block row J)
  __shared__ double cred[4][T][4];
  for (int i = threadIdx.x; i < 2 * T; i += 256) {
    const int R = (i < T ? I * T + i : J * T + i - T);
    const bool in = R < n;
    double* d = i < T ? xr[i] : xk[i - T];
    d[0] = in ? xD[2 * int64_t(R)] : 0.0;
    d[1] = in ? xD[2 * int64_t(R) + 1] : 0.0;
    d[2] = in ? xN[2 * int64_t(R)] : 0.0;
    d[3] = in ? xN[2 * int64_t(R) + 1] : 0.0;
  }
  double ca[NU][2][4];
#pragma unroll
  for (int k = 0; k < NU; ++k)
#pragma unroll
    for (int u = 0; u < 2; ++u) ca[k][u][0] = ca[k][u][1] = ca[k][u][2] = ca[k][u][3] = 0.0;
  const V* base = reinterpret_cast<const V*>(P) + int64_t(t) * 3 * MATV;
  __syncthreads();
  double xc[XREG ? NU : 1][2][4];
  if constexpr (XREG) {
#pragma unroll
    for (int k = 0; k < NU; ++k)
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q) xc[k][u][q] = xk[2 * (cl + LPR * k) + u][q];
  }
  for (int s = 0; s < RW / (G * RPS); ++s) {
    // column x values are re-read from LDS every step rather than held in
    // registers across the loop
    if constexpr (!XREG) asm volatile("" ::: "memory");
    const int r0 = wv * RW + G * RPS * s + g;
    V cv[RPS][NU], av[RPS][NU], bv[RPS][NU];
#pragma unroll
    for (int j = 0; j < RPS; ++j) {
      const V* rc = base + int64_t(r0 + G * j) * (3 * T / 2) + cl;
#pragma unroll
      for (int k = 0; k < NU; ++k) {
        cv[j][k] = __builtin_nontemporal_load(rc + LPR * k);
        av[j][k] = __builtin_nontemporal_load(rc + T / 2 + LPR * k);
        bv[j][k] = __builtin_nontemporal_load(rc + T + LPR * k);
      }
    }
    double a[RPS][4];
#pragma unroll
    for (int j = 0; j < RPS; ++j) {
      const int r = r0 + G * j;
      const double dr = xr[r][0], di = xr[r][1], nr = xr[r][2], ni = xr[r][3];
      a[j][0] = a[j][1] = a[j][2] = a[j][3] = 0.0;
#pragma unroll
      for (int k = 0; k < NU; ++k)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const double cr = double(cv[j][k][2 * u]), ci = double(cv[j][k][2 * u + 1]);
          const double sr = double(av[j][k][2 * u]), si = double(av[j][k][2 * u + 1]);
          const double tr = double(bv[j][k][2 * u]), ti = double(bv[j][k][2 * u + 1]);
          const double* xq = XREG ? xc[XREG ? k : 0][u] : xk[2 * (cl + LPR * k) + u];
          const double xdr = xq[0], xdi = xq[1], xnr = xq[2], xni = xq[3];
          // chains of fused multiply-adds (four per accumulator and entry)
          a[j][0] = fma(-si, xni, fma(sr, xnr, fma(-ci, xdi, fma(cr, xdr, a[j][0]))));
          a[j][1] = fma(si, xnr, fma(sr, xni, fma(ci, xdr, fma(cr, xdi, a[j][1]))));
          a[j][2] = fma(-ti, xdi, fma(tr, xdr, fma(-ci, xni, fma(cr, xnr, a[j][2]))));
          a[j][3] = fma(ti, xdr, fma(tr, xdi, fma(ci, xnr, fma(cr, xni, a[j][3]))));
          ca[k][u][0] = fma(-si, ni, fma(sr, nr, fma(-ci, di, fma(cr, dr, ca[k][u][0]))));
          ca[k][u][1] = fma(si, nr, fma(sr, ni, fma(ci, dr, fma(cr, di, ca[k][u][1]))));
          ca[k][u][2] = fma(-ti, di, fma(tr, dr, fma(-ci, ni, fma(cr, nr, ca[k][u][2]))));
          ca[k][u][3] = fma(ti, dr, fma(tr, di, fma(ci, nr, fma(cr, ni, ca[k][u][3]))));
        }
    }
#pragma unroll
    for (int j = 0; j < RPS; ++j) {
#pragma unroll
      for (int q = 0; q < 4; ++q) a[j][q] = row_sum<LPR>(a[j][q]);
      if (cl == 0) {
        double* p = part + ((int64_t(I) * nt + J) * T + r0 + G * j) * 4;
        p[0] = a[j][0];
        p[1] = a[j][1];
        p[2] = a[j][2];
        p[3] = a[j][3];
      }
    }
  }
  if (I == J) return;  // uniform per workgroup; the diagonal tile is whole and gives row sums only
#pragma unroll
  for (int k = 0; k < NU; ++k)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double v = ca[k][u][q];
#pragma unroll
        for (int o = LPR; o < 64; o <<= 1) v += __shfl_xor(v, o, WAVE);
        if (g == 0) cred[wv][2 * (cl + LPR * k) + u][q] = v;
      }
  __syncthreads();
  double* p = part + (int64_t(J) * nt + I) * T * 4;
  for (int i = threadIdx.x; i < T * 4; i += 256) {
    const int c = i >> 2, q = i & 3;
    p[i] = ((cred[0][c][q] + cred[1][c][q]) + cred[2][c][q]) + cred[3][c][q];
  }
}

// y = sum of the partial slots of each row plus the correction row.  A
// workgroup takes 16 rows; thread (q, r) (r fastest: consecutive threads read
// consecutive rows of a slot) adds slots q, q + 16, ... and correction entries
// q, q + 16, ... of its row, then the 16 sums are added in q order.
template <typename M, int T>
__global__ __launch_bounds__(256) void k_sym_reduce(const double* __restrict__ part, int nt, int n,
                                                    const int64_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ col, const M* __restrict__ val,
                                                    const double* __restrict__ xD, const double* __restrict__ xN,
                                                    double* __restrict__ yD, double* __restrict__ yN) {
  const int rr = threadIdx.x & 15, qq = threadIdx.x >> 4;
  const int R = blockIdx.x * 16 + rr;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (R < n) {
    const int K = R / T, r = R - K * T;
    for (int s = qq; s < nt; s += 16) {
      const d4v v = *reinterpret_cast<const d4v*>(part + ((int64_t(K) * nt + s) * T + r) * 4);
      a0 += v[0];
      a1 += v[1];
      a2 += v[2];
      a3 += v[3];
    }
    for (int64_t k = rowptr[R] + qq; k < rowptr[R + 1]; k += 16) {
      const int64_t c = col[k];
      const double dr = xD[2 * c], di = xD[2 * c + 1], nr = xN[2 * c], ni = xN[2 * c + 1];
      const M* v = val + 6 * k;
      const double cr = v[0], ci = v[1], sr = v[2], si = v[3], tr = v[4], ti = v[5];
      a0 += cr * dr - ci * di + sr * nr - si * ni;
      a1 += cr * di + ci * dr + sr * ni + si * nr;
      a2 += cr * nr - ci * ni + tr * dr - ti * di;
      a3 += cr * ni + ci * nr + tr * di + ti * dr;
    }
  }
  __shared__ double red[16][16][4];
  red[qq][rr][0] = a0;
  red[qq][rr][1] = a1;
  red[qq][rr][2] = a2;
  red[qq][rr][3] = a3;
  __syncthreads();
  if (qq == 0 && R < n) {
    double o[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int p = 0; p < 16; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) o[q] += red[p][rr][q];
    yD[2 * int64_t(R)] = o[0];
    yD[2 * int64_t(R) + 1] = o[1];
    yN[2 * int64_t(R)] = o[2];
    yN[2 * int64_t(R) + 1] = o[3];
  }
}

template <typename M>
void launch_pack_sym3(const M* Se, const M* Ce, const M* Si, const M* Ci, int64_t ld, int n, const int32_t* tij,
                      int64_t ntiles, double ke, double kir, double kii, M* P, hipStream_t st) {
  const int64_t blocks = ntiles * SYM_T * SYM_T / 256;
  hipLaunchKernelGGL((k_pack_sym3<M, SYM_T>), dim3(unsigned(blocks)), dim3(256), 0, st, Se, Ce, Si, Ci, ld, n, tij,
                     ke, kir, kii, P);
}

template <typename M>
void launch_sym_corr(const M* Se, const M* Ce, const M* Si, const M* Ci, int64_t ld, const int32_t* crow,
                     const int32_t* col, int64_t nnz, double ke, double kir, double kii, M* val, hipStream_t st) {
  if (nnz == 0) return;
  hipLaunchKernelGGL((k_sym_corr<M>), dim3(unsigned((nnz + 255) / 256)), dim3(256), 0, st, Se, Ce, Si, Ci, ld, crow,
                     col, nnz, ke, kir, kii, val);
}

template <typename M>
void launch_gemv_sym3(const M* P, const int32_t* tij, int64_t ntiles, int nt, int n, const double* xD,
                      const double* xN, double* part, hipStream_t st) {
  // measured on the 7680-edge operator: FP32 best with 32 lanes per row and
  // the column x values in registers, FP64 with 16 lanes per row
  if constexpr (sizeof(M) == 4)
    hipLaunchKernelGGL((k_gemv_sym3<M, SYM_T, 32, 1, 1, true>), dim3(unsigned(ntiles)), dim3(256), 0, st, P, tij, nt,
                       n, xD, xN, part);
  else
    hipLaunchKernelGGL((k_gemv_sym3<M, SYM_T, 16, 1, 1, false>), dim3(unsigned(ntiles)), dim3(256), 0, st, P, tij,
                       nt, n, xD, xN, part);
}

template <typename M>
void launch_sym_reduce(const double* part, int nt, int n, const int64_t* rowptr, const int32_t* col, const M* val,
                       const double* xD, const double* xN, double* yD, double* yN, hipStream_t st) {
  hipLaunchKernelGGL((k_sym_reduce<M, SYM_T>), dim3(unsigned((n + 15) / 16)), dim3(256), 0, st, part, nt, n, rowptr,
                     col, val, xD, xN, yD, yN);
}

template void launch_sym_corr_sing<float>(const int64_t*, const int32_t*, const double*, int64_t, double, double,
                                          double, float*, hipStream_t);
template void launch_sym_corr_sing<double>(const int64_t*, const int32_t*, const double*, int64_t, double, double,
                                           double, double*, hipStream_t);
template void launch_mirror_lower<float>(float*, int64_t, int, const int32_t*, const int32_t*, const int64_t*,
                                         const int32_t*, const double*, int64_t, int, hipStream_t);
template void launch_mirror_lower<double>(double*, int64_t, int, const int32_t*, const int32_t*, const int64_t*,
                                          const int32_t*, const double*, int64_t, int, hipStream_t);

#define PMCHWT_SYM_INST(M)                                                                                          \
  template void launch_pack_sym3<M>(const M*, const M*, const M*, const M*, int64_t, int, const int32_t*, int64_t, \
                                    double, double, double, M*, hipStream_t);                                      \
  template void launch_sym_corr<M>(const M*, const M*, const M*, const M*, int64_t, const int32_t*, const int32_t*, \
                                   int64_t, double, double, double, M*, hipStream_t);                              \
  template void launch_gemv_sym3<M>(const M*, const int32_t*, int64_t, int, int, const double*, const double*,      \
                                    double*, hipStream_t);                                                          \
  template void launch_sym_reduce<M>(const double*, int, int, const int64_t*, const int32_t*, const M*,            \
                                     const double*, const double*, double*, double*, hipStream_t);
PMCHWT_SYM_INST(float)
PMCHWT_SYM_INST(double)
#undef PMCHWT_SYM_INST

template <typename M>
void launch_gemv_pmchwt(const M* S, const M* C, int64_t ld, int rows, int cols, double kr, double ki,
                        const double* xD, const double* xN, double* yD, double* yN, int nrhs, int64_t vstride,
                        hipStream_t st) {
  auto grid = [rows](int rpw) { return dim3(unsigned((rows + 4 * rpw - 1) / (4 * rpw))); };
  const dim3 block(256);
  int r0 = 0;
  while (r0 < nrhs) {
    const int left = nrhs - r0;
    const double* xd = xD + 2 * int64_t(r0) * vstride;
    const double* xn = xN + 2 * int64_t(r0) * vstride;
    double* yd = yD + 2 * int64_t(r0) * vstride;
    double* yn = yN + 2 * int64_t(r0) * vstride;
    if (left >= 4) {
      hipLaunchKernelGGL((k_gemv_pmchwt<M, 4>), grid(GemvRows<M, 4>::value), block, 0, st, S, C, ld, rows, cols, kr,
                         ki, xd, xn, yd, yn, vstride);
      r0 += 4;
    } else if (left >= 2) {
      hipLaunchKernelGGL((k_gemv_pmchwt<M, 2>), grid(GemvRows<M, 2>::value), block, 0, st, S, C, ld, rows, cols, kr,
                         ki, xd, xn, yd, yn, vstride);
      r0 += 2;
    } else {
      hipLaunchKernelGGL((k_gemv_pmchwt<M, 1>), grid(GemvRows<M, 1>::value), block, 0, st, S, C, ld, rows, cols, kr,
                         ki, xd, xn, yd, yn, vstride);
      r0 += 1;
    }
  }
}
template void launch_gemv_pmchwt<double>(const double*, const double*, int64_t, int, int, double, double,
                                         const double*, const double*, double*, double*, int, int64_t,
                                         hipStream_t);
template void launch_gemv_pmchwt<float>(const float*, const float*, int64_t, int, int, double, double,
                                        const double*, const double*, double*, double*, int, int64_t,
                                        hipStream_t);

// ---------------------------------------------------------------------------
// Same block structure on a CSR pattern; S or C may be null (HS / HC: which
// are present, so that only their sums are formed and reduced).  32 lanes per
// row, two rows per wavefront: the near-field rows hold 100-300 entries.
// ---------------------------------------------------------------------------
template <typename M, int NR, bool HS, bool HC>
__global__ __launch_bounds__(256) void k_spmv_pmchwt(const int64_t* __restrict__ rowptr,
                                                     const int32_t* __restrict__ col, const M* __restrict__ S,
                                                     const M* __restrict__ C, int rows, double kr, double ki,
                                                     const double* __restrict__ xD,
                                                     const double* __restrict__ xN, double* yD, double* yN,
                                                     int64_t vstride, int acc) {
  // right-hand sides NR blockIdx.y .. NR blockIdx.y + NR - 1
  const int64_t g0 = 2 * int64_t(blockIdx.y) * NR * vstride;
  xD += g0;
  xN += g0;
  yD += g0;
  yN += g0;
  const int lane = threadIdx.x & 31;
  const int row = blockIdx.x * (blockDim.x / 32) + threadIdx.x / 32;
  const bool live = row < rows;  // both halves of a wavefront take part in the shuffles
  double a[NR][8];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int q = 0; q < 8; ++q) a[r][q] = 0.0;
  const int64_t p0 = live ? rowptr[row] : 0, p1 = live ? rowptr[row + 1] : 0;
  // unrolled so that the index and value loads of later entries are in
  // flight while earlier ones gather x (the sum per lane stays in order)
#pragma unroll 4
  for (int64_t p = p0 + lane; p < p1; p += 32) {
    const int j = col[p];
    double sr = 0, si = 0, cr = 0, ci = 0;
    if (HS) {
      sr = double(S[2 * p]);
      si = double(S[2 * p + 1]);
    }
    if (HC) {
      cr = double(C[2 * p]);
      ci = double(C[2 * p + 1]);
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double* pd = xD + 2 * (int64_t(r) * vstride + j);
      const double* pn = xN + 2 * (int64_t(r) * vstride + j);
      const double dr = pd[0], di = pd[1], nr = pn[0], ni = pn[1];
      if (HC) {
        a[r][0] += cr * dr - ci * di;
        a[r][1] += cr * di + ci * dr;
        a[r][6] += cr * nr - ci * ni;
        a[r][7] += cr * ni + ci * nr;
      }
      if (HS) {
        a[r][2] += sr * nr - si * ni;
        a[r][3] += sr * ni + si * nr;
        a[r][4] += sr * dr - si * di;
        a[r][5] += sr * di + si * dr;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const bool used = (q >= 2 && q < 6) ? HS : HC;
      if (!used) continue;
      double v = a[r][q];
#pragma unroll
      for (int o = 16; o >= 1; o >>= 1) v += __shfl_xor(v, o, WAVE);
      a[r][q] = v;
    }
  if (live && lane == 0) {
    const double k2 = kr * kr + ki * ki;
    const double ikr = kr / k2, iki = -ki / k2;
    for (int r = 0; r < NR; ++r) {
      double* yd = yD + 2 * (int64_t(r) * vstride + row);
      double* yn = yN + 2 * (int64_t(r) * vstride + row);
      const double t_re = a[r][2] * ikr - a[r][3] * iki, t_im = a[r][2] * iki + a[r][3] * ikr;
      const double u_re = -(kr * a[r][4] - ki * a[r][5]), u_im = -(kr * a[r][5] + ki * a[r][4]);
      const double o0 = acc ? yd[0] : 0.0, o1 = acc ? yd[1] : 0.0, o2 = acc ? yn[0] : 0.0, o3 = acc ? yn[1] : 0.0;
      yd[0] = o0 + (a[r][0] + t_re);
      yd[1] = o1 + (a[r][1] + t_im);
      yn[0] = o2 + (u_re + a[r][6]);
      yn[1] = o3 + (u_im + a[r][7]);
    }
  }
}

template <typename M, int NR>
static void spmv_pmchwt_launch(dim3 grid, const int64_t* rowptr, const int32_t* col, const M* S, const M* C, int rows,
                               double kr, double ki, const double* xd, const double* xn, double* yd, double* yn,
                               int64_t vstride, bool acc, hipStream_t st) {
  if (S && C)
    hipLaunchKernelGGL((k_spmv_pmchwt<M, NR, true, true>), grid, dim3(256), 0, st, rowptr, col, S, C, rows, kr, ki,
                       xd, xn, yd, yn, vstride, int(acc));
  else if (S)
    hipLaunchKernelGGL((k_spmv_pmchwt<M, NR, true, false>), grid, dim3(256), 0, st, rowptr, col, S, C, rows, kr, ki,
                       xd, xn, yd, yn, vstride, int(acc));
  else if (C)
    hipLaunchKernelGGL((k_spmv_pmchwt<M, NR, false, true>), grid, dim3(256), 0, st, rowptr, col, S, C, rows, kr, ki,
                       xd, xn, yd, yn, vstride, int(acc));
  else
    hipLaunchKernelGGL((k_spmv_pmchwt<M, NR, false, false>), grid, dim3(256), 0, st, rowptr, col, S, C, rows, kr, ki,
                       xd, xn, yd, yn, vstride, int(acc));
}

// groups of 4 right-hand sides in one launch (grid.y over the groups), the
// remainder one at a time in a second launch
template <typename M>
void launch_spmv_pmchwt(const int64_t* rowptr, const int32_t* col, const M* S, const M* C, int rows, double kr,
                        double ki, const double* xD, const double* xN, double* yD, double* yN, int nrhs,
                        int64_t vstride, hipStream_t st, bool acc) {
  const unsigned gx = unsigned((rows + 7) / 8);
  const int n4 = nrhs / 4, r0 = 4 * n4;
  if (n4 > 0)
    spmv_pmchwt_launch<M, 4>(dim3(gx, unsigned(n4)), rowptr, col, S, C, rows, kr, ki, xD, xN, yD, yN, vstride, acc,
                             st);
  if (nrhs > r0) {
    const int64_t o = 2 * int64_t(r0) * vstride;
    spmv_pmchwt_launch<M, 1>(dim3(gx, unsigned(nrhs - r0)), rowptr, col, S, C, rows, kr, ki, xD + o, xN + o, yD + o,
                             yN + o, vstride, acc, st);
  }
}
template void launch_spmv_pmchwt<double>(const int64_t*, const int32_t*, const double*, const double*, int,
                                         double, double, const double*, const double*, double*, double*, int,
                                         int64_t, hipStream_t, bool);
template void launch_spmv_pmchwt<float>(const int64_t*, const int32_t*, const float*, const float*, int, double,
                                        double, const double*, const double*, double*, double*, int, int64_t,
                                        hipStream_t, bool);

// ---------------------------------------------------------------------------
// y = alpha * M x, M real dense row-major; complex vectors (overwrites y).
// ---------------------------------------------------------------------------
template <int NR>
__global__ __launch_bounds__(256) void k_gemv_real(const double* __restrict__ Mat, int64_t ld, int rows, int cols,
                                                   double alpha, const double* __restrict__ x, double* y,
                                                   int64_t vstride) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (row >= rows) return;
  double a[NR][2];
  for (int r = 0; r < NR; ++r) a[r][0] = a[r][1] = 0.0;
  const double* mr = Mat + int64_t(row) * ld;
  for (int j = lane; j < cols; j += 64) {
    const double m = mr[j];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double* px = x + 2 * (int64_t(r) * vstride + j);
      a[r][0] += m * px[0];
      a[r][1] += m * px[1];
    }
  }
  for (int r = 0; r < NR; ++r) {
    a[r][0] = wsum(a[r][0]);
    a[r][1] = wsum(a[r][1]);
  }
  if (lane == 0)
    for (int r = 0; r < NR; ++r) {
      double* py = y + 2 * (int64_t(r) * vstride + row);
      py[0] = alpha * a[r][0];
      py[1] = alpha * a[r][1];
    }
}

void launch_gemv_real(const double* Mat, int64_t ld, int rows, int cols, double alpha, const double* x, double* y,
                      int nrhs, int64_t vstride, hipStream_t st) {
  const dim3 grid((rows + 3) / 4), block(256);
  for (int r0 = 0; r0 < nrhs;) {
    const int left = nrhs - r0;
    const double* xx = x + 2 * int64_t(r0) * vstride;
    double* yy = y + 2 * int64_t(r0) * vstride;
    if (left >= 8) {
      hipLaunchKernelGGL((k_gemv_real<8>), grid, block, 0, st, Mat, ld, rows, cols, alpha, xx, yy, vstride);
      r0 += 8;
    } else if (left >= 2) {
      hipLaunchKernelGGL((k_gemv_real<2>), grid, block, 0, st, Mat, ld, rows, cols, alpha, xx, yy, vstride);
      r0 += 2;
    } else {
      hipLaunchKernelGGL((k_gemv_real<1>), grid, block, 0, st, Mat, ld, rows, cols, alpha, xx, yy, vstride);
      r0 += 1;
    }
  }
}

__global__ void k_transpose(const double* in, double* out, int n) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const int i = by + k, j = bx + threadIdx.x;
    if (i < n && j < n) tile[k][threadIdx.x] = in[int64_t(i) * n + j];
  }
  __syncthreads();
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const int i = bx + k, j = by + threadIdx.x;
    if (i < n && j < n) out[int64_t(i) * n + j] = tile[threadIdx.x][k];
  }
}

void launch_transpose(const double* in, double* out, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_transpose, dim3((n + 31) / 32, (n + 31) / 32), dim3(32, 8), 0, st, in, out, n);
}

// ---------------------------------------------------------------------------
// Krylov helpers.  Vector i of right-hand side r: V + 2*(i*vstep + r*rstride_v).
// ---------------------------------------------------------------------------
__global__ void k_dots(const double* V, int64_t vstep, const double* w, int64_t wstride, int n,
                       const int32_t* active, int64_t rstride_v, double* out, int nvec) {
  const int i = blockIdx.x, r = blockIdx.y;
  if (!active[r]) return;
  const double* v = V + 2 * (int64_t(i) * vstep + int64_t(r) * rstride_v);
  const double* ww = w + 2 * int64_t(r) * wstride;
  double re = 0, im = 0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const double vr = v[2 * k], vi = v[2 * k + 1], xr = ww[2 * k], xi = ww[2 * k + 1];
    re += vr * xr + vi * xi;  // conj(v) w
    im += vr * xi - vi * xr;
  }
  __shared__ double sr[256], si[256];
  sr[threadIdx.x] = re;
  si[threadIdx.x] = im;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      si[threadIdx.x] += si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * (int64_t(r) * nvec + i)] = sr[0];
    out[2 * (int64_t(r) * nvec + i) + 1] = si[0];
  }
}

// Dots split over S chunks of the vector length (more workgroups than one per
// vector), partial sums part[((r nvec + i) S + s)], summed in a fixed order.
__global__ void k_dots_part(const double* V, int64_t vstep, const double* w, int64_t wstride, int n,
                            const int32_t* active, int64_t rstride_v, double* part, int nvec, int S, int chunk) {
  const int i = blockIdx.x, sidx = blockIdx.y, r = blockIdx.z;
  double* o = part + 2 * ((int64_t(r) * nvec + i) * S + sidx);
  if (!active[r]) {
    if (threadIdx.x == 0) o[0] = o[1] = 0.0;
    return;
  }
  const double2* v = reinterpret_cast<const double2*>(V) + int64_t(i) * vstep + int64_t(r) * rstride_v;
  const double2* ww = reinterpret_cast<const double2*>(w) + int64_t(r) * wstride;
  const int k0 = sidx * chunk, k1 = min(n, k0 + chunk);
  double re = 0, im = 0;
#pragma unroll 4
  for (int k = k0 + threadIdx.x; k < k1; k += blockDim.x) {
    const double2 a = v[k], x = ww[k];
    re += a.x * x.x + a.y * x.y;
    im += a.x * x.y - a.y * x.x;
  }
  // wavefront sums, then the four wavefronts in order
  re = wsum(re);
  im = wsum(im);
  __shared__ double sr[4], si[4];
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sr[wv] = re;
    si[wv] = im;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    o[0] = ((sr[0] + sr[1]) + sr[2]) + sr[3];
    o[1] = ((si[0] + si[1]) + si[2]) + si[3];
  }
}

int dots_splits(int nvec, int nrhs, int n) {
  const int want = (1024 + nvec * nrhs - 1) / (nvec * nrhs);
  return std::max(1, std::min({want, 64, (n + 255) / 256}));
}

int dots_part_only(const double* V, int64_t vstep, int nvec, const double* w, int64_t wstride, int n,
                   const int32_t* active, int nrhs, int64_t rstride_v, double* part, hipStream_t st) {
  const int S = dots_splits(nvec, nrhs, n);
  if (S == 1) {
    hipLaunchKernelGGL(k_dots, dim3(nvec, nrhs), dim3(256), 0, st, V, vstep, w, wstride, n, active, rstride_v, part,
                       nvec);
  } else {
    const int chunk = (n + S - 1) / S;
    hipLaunchKernelGGL(k_dots_part, dim3(nvec, S, nrhs), dim3(256), 0, st, V, vstep, w, wstride, n, active,
                       rstride_v, part, nvec, S, chunk);
  }
  return S;
}

// w^r[k] += sign * sum_i V_i^r[k] h[r][i], where each coefficient is the sum
// of S partial values, h[r][i] = sum_s hp[(r hstride + i) S + s] (complex),
// added in the order s = 0, 1, ... (S = 1: the coefficients themselves).  A
// workgroup owns 64 consecutive elements; the coefficients of up to 1024
// vectors at a time are summed into LDS, then its UPD_WAVES wavefronts take
// every UPD_WAVES-th vector (coalesced 1 KB reads per vector, four loads in
// flight each: with one workgroup per 64 elements there are only n / 64
// workgroups, so the wavefronts of one are what fills the CU) and the partial
// results are added in a fixed order through LDS.
// With nrm2 given, the workgroup also stores the sum of |w|^2 over its 64
// updated elements at nrm2[r gridDim.x + blockIdx.x] (0 for an inactive
// right-hand side): the partial sums of the new vector's norm.
constexpr int UPD_WAVES = 16;
__global__ __launch_bounds__(64 * UPD_WAVES) void k_update(const double* V, int64_t vstep, int nvec, double* w,
                                                           int64_t wstride, int n, const int32_t* active,
                                                           int64_t rstride_v, const double* hp, int64_t hstride,
                                                           int S, double sign, double* nrm2) {
  constexpr int CH = 1024;
  const int r = blockIdx.y;
  if (!active[r]) {
    if (nrm2 && threadIdx.x == 0) nrm2[int64_t(r) * gridDim.x + blockIdx.x] = 0.0;
    return;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int k = blockIdx.x * 64 + lane;
  const bool in = k < n;
  const int kk = in ? k : n - 1;
  const double2* base = reinterpret_cast<const double2*>(V) + int64_t(r) * rstride_v + kk;
  const double2* hr_ = reinterpret_cast<const double2*>(hp) + int64_t(r) * hstride * S;
  __shared__ double2 hs[CH];
  __shared__ double2 part[UPD_WAVES - 1][64];
  double re = 0, im = 0;
  for (int i0 = 0; i0 < nvec; i0 += CH) {
    const int nc = min(CH, nvec - i0);
    __syncthreads();
    for (int t = threadIdx.x; t < nc; t += blockDim.x) {
      double2 h = {0.0, 0.0};
      // unrolled: the partial sums' loads in flight together (added in order)
#pragma unroll 8
      for (int sidx = 0; sidx < S; ++sidx) {
        const double2 v = hr_[int64_t(i0 + t) * S + sidx];
        h.x += v.x;
        h.y += v.y;
      }
      hs[t] = h;
    }
    __syncthreads();
    const double2* bi = base + int64_t(i0) * vstep;
    int i = wv;
    for (; i + 3 * UPD_WAVES < nc; i += 4 * UPD_WAVES) {
      double2 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = bi[int64_t(i + UPD_WAVES * u) * vstep];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double2 h = hs[i + UPD_WAVES * u];
        re += v[u].x * h.x - v[u].y * h.y;
        im += v[u].x * h.y + v[u].y * h.x;
      }
    }
    for (; i < nc; i += UPD_WAVES) {
      const double2 v = bi[int64_t(i) * vstep];
      const double2 h = hs[i];
      re += v.x * h.x - v.y * h.y;
      im += v.x * h.y + v.y * h.x;
    }
  }
  if (wv > 0) part[wv - 1][lane] = double2{re, im};
  __syncthreads();
  if (wv == 0) {
    double sq = 0.0;
    if (in) {
#pragma unroll
      for (int q = 0; q < UPD_WAVES - 1; ++q) {
        re += part[q][lane].x;
        im += part[q][lane].y;
      }
      double* ww = w + 2 * (int64_t(r) * wstride + k);
      const double nr = ww[0] + sign * re, ni = ww[1] + sign * im;
      ww[0] = nr;
      ww[1] = ni;
      sq = nr * nr + ni * ni;
    }
    if (nrm2) {
      sq = wsum(sq);
      if (lane == 0) nrm2[int64_t(r) * gridDim.x + blockIdx.x] = sq;
    }
  }
}

int update_blocks(int n) { return (n + 63) / 64; }

void launch_update(const double* V, int64_t vstep, int nvec, double* w, int64_t wstride, int n,
                   const int32_t* active, int nrhs, int64_t rstride_v, const double* h, int64_t hstride, double sign,
                   hipStream_t st, int S, double* nrm2) {
  hipLaunchKernelGGL(k_update, dim3(update_blocks(n), nrhs), dim3(64 * UPD_WAVES), 0, st, V, vstep, nvec, w, wstride, n, active,
                     rstride_v, h, hstride, S, sign, nrm2);
}

__global__ void k_norms(const double* w, int64_t wstride, int n, double* out) {
  const int r = blockIdx.x;
  const double* ww = w + 2 * int64_t(r) * wstride;
  double s = 0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) s += ww[2 * k] * ww[2 * k] + ww[2 * k + 1] * ww[2 * k + 1];
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int q = blockDim.x / 2; q > 0; q >>= 1) {
    if (threadIdx.x < q) red[threadIdx.x] += red[threadIdx.x + q];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[r] = sqrt(red[0]);
}

__global__ void k_norms_part(const double* w, int64_t wstride, int n, int S, int chunk, double* part) {
  const int sidx = blockIdx.x, r = blockIdx.y;
  const double* ww = w + 2 * int64_t(r) * wstride;
  const int k0 = sidx * chunk, k1 = min(n, k0 + chunk);
  double s = 0;
  for (int k = k0 + threadIdx.x; k < k1; k += blockDim.x) s += ww[2 * k] * ww[2 * k] + ww[2 * k + 1] * ww[2 * k + 1];
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int q = blockDim.x / 2; q > 0; q >>= 1) {
    if (threadIdx.x < q) red[threadIdx.x] += red[threadIdx.x + q];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[int64_t(r) * S + sidx] = red[0];
}

__global__ void k_norms_fin(const double* part, int S, int nrhs, double* out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  double s = 0;
  for (int sidx = 0; sidx < S; ++sidx) s += part[int64_t(r) * S + sidx];
  out[r] = sqrt(s);
}

int norm_splits(int nrhs, int n) { return std::max(1, std::min({(256 + nrhs - 1) / nrhs, 64, (n + 255) / 256})); }

void launch_norms(const double* w, int64_t wstride, int n, int nrhs, double* out, hipStream_t st, double* part) {
  const int S = part ? norm_splits(nrhs, n) : 1;
  if (S == 1) {
    hipLaunchKernelGGL(k_norms, dim3(nrhs), dim3(256), 0, st, w, wstride, n, out);
    return;
  }
  const int chunk = (n + S - 1) / S;
  hipLaunchKernelGGL(k_norms_part, dim3(S, nrhs), dim3(256), 0, st, w, wstride, n, S, chunk, part);
  hipLaunchKernelGGL(k_norms_fin, dim3((nrhs + 255) / 256), dim3(256), 0, st, part, S, nrhs, out);
}

__global__ void k_scale_copy(const double* w, int64_t wstride, double* v, int64_t vstride, int n,
                             const double* scale) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (k >= n) return;
  const double s = scale[r];
  v[2 * (int64_t(r) * vstride + k)] = s * w[2 * (int64_t(r) * wstride + k)];
  v[2 * (int64_t(r) * vstride + k) + 1] = s * w[2 * (int64_t(r) * wstride + k) + 1];
}

void launch_scale_copy(const double* w, int64_t wstride, double* v, int64_t vstride, int n, int nrhs,
                       const double* scale, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_copy, dim3((n + 255) / 256, nrhs), dim3(256), 0, st, w, wstride, v, vstride, n, scale);
}

// End of an Arnoldi step on the device: v = w / |w| per right-hand side (0
// where inactive or |w| = 0), |w|^2 the sum of S2 partial values.  The first
// workgroup of each right-hand side also finishes the two projection passes'
// split sums (S1 partials per coefficient, nvec coefficients) and the norm
// into fin = [h1 (nvec nrhs complex) | h2 (same) | |w| (nrhs)] for the host,
// every sum taken in order of the partial index as the update kernels do.
__global__ void k_finish_step(const double* w, int64_t wstride, double* v, int64_t vstride, int n,
                              const double* nrm2, int S2, const int32_t* active, const double* h1p,
                              const double* h2p, int S1, int nvec, int nrhs, double* fin, double* flags,
                              double seq) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  // |w|^2 from its partial sums: strided per thread, then a fixed tree over
  // the workgroup (the same order in every workgroup)
  __shared__ double red[256];
  double ss = 0;
  for (int sidx = threadIdx.x; sidx < S2; sidx += blockDim.x) ss += nrm2[int64_t(r) * S2 + sidx];
  red[threadIdx.x] = ss;
  __syncthreads();
  for (int q = blockDim.x / 2; q > 0; q >>= 1) {
    if (threadIdx.x < q) red[threadIdx.x] += red[threadIdx.x + q];
    __syncthreads();
  }
  const double h = sqrt(red[0]);
  if (blockIdx.x == 0) {
    const double2* p1 = reinterpret_cast<const double2*>(h1p) + int64_t(r) * nvec * S1;
    const double2* p2 = reinterpret_cast<const double2*>(h2p) + int64_t(r) * nvec * S1;
    double2* f1 = reinterpret_cast<double2*>(fin) + int64_t(r) * nvec;
    double2* f2 = reinterpret_cast<double2*>(fin) + int64_t(nrhs) * nvec + int64_t(r) * nvec;
    for (int i = threadIdx.x; i < nvec; i += blockDim.x) {
      double2 a = {0.0, 0.0}, b = {0.0, 0.0};
#pragma unroll 8
      for (int sidx = 0; sidx < S1; ++sidx) {
        const double2 u = p1[int64_t(i) * S1 + sidx], t = p2[int64_t(i) * S1 + sidx];
        a.x += u.x;
        a.y += u.y;
        b.x += t.x;
        b.y += t.y;
      }
      f1[i] = a;
      f2[i] = b;
    }
    if (threadIdx.x == 0) fin[4 * int64_t(nrhs) * nvec + r] = h;
    // the step number after the values, once they are visible to the host
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) *reinterpret_cast<volatile double*>(flags + r) = seq;
  }
  if (k >= n) return;
  const double s = (active[r] && h > 0) ? 1.0 / h : 0.0;
  v[2 * (int64_t(r) * vstride + k)] = s * w[2 * (int64_t(r) * wstride + k)];
  v[2 * (int64_t(r) * vstride + k) + 1] = s * w[2 * (int64_t(r) * wstride + k) + 1];
}

void launch_finish_step(const double* w, int64_t wstride, double* v, int64_t vstride, int n, int nrhs,
                        const double* nrm2, int S2, const int32_t* active, const double* h1p, const double* h2p,
                        int S1, int nvec, double* fin, double* flags, double seq, hipStream_t st) {
  hipLaunchKernelGGL(k_finish_step, dim3((n + 255) / 256, nrhs), dim3(256), 0, st, w, wstride, v, vstride, n, nrm2,
                     S2, active, h1p, h2p, S1, nvec, nrhs, fin, flags, seq);
}

// API layout (scatterer-major [D_m ; N_m] per right-hand side, complex) <->
// internal layout ([D ; N] over the union): one thread per (rhs, component,
// union edge); soff: the scatterers' edge offsets (nsc + 1 entries, last E).
__global__ void k_layout(const double* __restrict__ in, double* __restrict__ out, int nrhs, int E,
                         const int32_t* __restrict__ soff, int nsc, int to_internal) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t per = 2 * int64_t(E);
  if (t >= per * nrhs) return;
  const int64_t r = t / per;
  const int rem = int(t - r * per), comp = rem / E, e = rem - comp * E;
  int lo = 0, hi = nsc;  // the last scatterer whose first edge is <= e
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (soff[mid] <= e)
      lo = mid;
    else
      hi = mid;
  }
  const int o = soff[lo], Em = soff[lo + 1] - o;
  const int64_t ki = r * per + int64_t(comp) * E + e;
  const int64_t ka = r * per + 2 * int64_t(o) + int64_t(comp) * Em + (e - o);
  const int64_t src = to_internal ? ka : ki, dst = to_internal ? ki : ka;
  out[2 * dst] = in[2 * src];
  out[2 * dst + 1] = in[2 * src + 1];
}

void launch_layout(const double* in, double* out, int nrhs, int E, const int32_t* soff, int nsc, bool to_internal,
                   hipStream_t st) {
  const int64_t n = 2 * int64_t(E) * nrhs;
  if (n > 0)
    hipLaunchKernelGGL(k_layout, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, in, out, nrhs, E, soff, nsc,
                       int(to_internal));
}

// y = a y + b x  (complex vectors, real scalars)
__global__ void k_axpby(double* y, const double* x, int64_t stride, int n, double a, double b) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (k >= 2 * int64_t(n)) return;
  const int64_t o = 2 * int64_t(r) * stride + k;
  y[o] = a * y[o] + b * x[o];
}

// rows [0, rows) of both components: element k < 4 rows (re/im, D/N)
__global__ void k_axpby_rows(double* y, const double* x, int64_t vstride, int rows, int64_t cstride, double a,
                             double b) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (k >= 4 * int64_t(rows)) return;
  const int64_t part = k / (2 * int64_t(rows)), w = k - part * 2 * int64_t(rows);
  const int64_t o = 2 * (int64_t(r) * vstride + part * cstride) + w;
  y[o] = a * y[o] + b * x[o];
}

void launch_axpby_rows(double* y, const double* x, int64_t vstride, int rows, int64_t cstride, int nrhs, double a,
                       double b, hipStream_t st) {
  hipLaunchKernelGGL(k_axpby_rows, dim3(unsigned((4 * int64_t(rows) + 255) / 256), nrhs), dim3(256), 0, st, y, x,
                     vstride, rows, cstride, a, b);
}

void launch_axpby(double* y, const double* x, int64_t stride, int n, int nrhs, double a, double b, hipStream_t st) {
  hipLaunchKernelGGL(k_axpby, dim3(unsigned((2 * int64_t(n) + 255) / 256), nrhs), dim3(256), 0, st, y, x, stride, n,
                     a, b);
}

template <typename T>
__global__ void k_zero(T* p, int64_t n) {
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += int64_t(gridDim.x) * blockDim.x)
    p[k] = T(0);
}

void launch_zero(double* p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_zero<double>, dim3(unsigned(blocks)), dim3(256), 0, st, p, n);
}

void launch_zero_f(float* p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_zero<float>, dim3(unsigned(blocks)), dim3(256), 0, st, p, n);
}

// complex vectors (nvec, each E long, stride sstride complex) <-> real
// column-major matrix E x 2 nvec (re, im columns), for LAPACK-style solves.
__global__ void k_pack(const double* src, int64_t sstride, int E, int nvec, double* dst) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= int64_t(E) * nvec) return;
  const int q = int(k / E), e = int(k % E);
  dst[int64_t(2 * q) * E + e] = src[2 * (int64_t(q) * sstride + e)];
  dst[int64_t(2 * q + 1) * E + e] = src[2 * (int64_t(q) * sstride + e) + 1];
}

__global__ void k_unpack(const double* src, int E, int nvec, double* dst, int64_t dstride) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= int64_t(E) * nvec) return;
  const int q = int(k / E), e = int(k % E);
  dst[2 * (int64_t(q) * dstride + e)] = src[int64_t(2 * q) * E + e];
  dst[2 * (int64_t(q) * dstride + e) + 1] = src[int64_t(2 * q + 1) * E + e];
}

void launch_pack_cols(const double* src, int64_t sstride, int E, int nvec, double* dst, hipStream_t st) {
  const int64_t n = int64_t(E) * nvec;
  hipLaunchKernelGGL(k_pack, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, src, sstride, E, nvec, dst);
}

void launch_unpack_cols(const double* src, int E, int nvec, double* dst, int64_t dstride, hipStream_t st) {
  const int64_t n = int64_t(E) * nvec;
  hipLaunchKernelGGL(k_unpack, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, src, E, nvec, dst, dstride);
}

}  // namespace pmchwt

namespace pmchwt {

// ---------------------------------------------------------------------------
// In-place inverse of a b x b column-major block (b <= 128) by Gauss-Jordan
// elimination without pivoting, one workgroup, block held in registers.  Used on
// the diagonal blocks of the blocked Gauss-Jordan inverse of the mixed mass
// matrix, whose symmetric part is positive definite (every leading block is
// safely invertible without row exchanges).
// ---------------------------------------------------------------------------
// Thread (ti, tj) of a 16 x 16 grid holds the 8 x 8 tile of rows 8 ti.. and
// columns 8 tj.. in registers.  Step k of the in-place Gauss-Jordan inverse
// is one rank-1 update
//   a_ij -= u_i v_j,  u_i = a_ik - [i == k],  v_j = a_kj / a_kk (j != k), v_k = 1 / a_kk,
// applied after column k has been reset to the unit vector e_k (checked
// entrywise: row k becomes a_kj / a_kk, column k becomes -a_ik / a_kk, the
// pivot 1 / a_kk).  The owners of column k+1 publish u for the next step and
// reset their registers; the owners of row k+1 publish that row; two LDS
// buffers alternate, so one barrier per step suffices.  Entries beyond b are
// padded with the identity and stay inert.
// Row k+1 and column k+1 are published by 16 threads with vector stores of 8
// values each, every thread reads 8 + 8 values per step, and with the pivot
// loop unrolled by 8 the register row / column of the next pivot is a
// compile-time index.  Padded steps beyond b (up to the next multiple of 8)
// act on identity rows and change nothing.
// Reciprocal of a pivot: the hardware reciprocal in FP32 (1 ulp; the FP32
// inverse only preconditions), the IEEE quotient in FP64
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

template <typename T, bool ROWMAJOR_OUT>
__global__ __launch_bounds__(256) void k_gj_block_inverse_t(const T* __restrict__ X, int64_t ldx,
                                                            T* __restrict__ out, int b) {
  constexpr int NB = 128;
  __shared__ T colk[2][NB], rowk[2][NB], pinv[2];
  const int t = threadIdx.x;
  const int ti = t >> 4, tj = t & 15;  // rows 8 ti .. +8, columns 8 tj .. +8
  const int r0 = 8 * ti, c0 = 8 * tj;
  T a[8][8];
#pragma unroll
  for (int r = 0; r < 8; ++r)
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int i = r0 + r, j = c0 + c;
      a[r][c] = (i < b && j < b) ? X[int64_t(j) * ldx + i] : T(i == j ? 1 : 0);
    }
  // publish row 0 and column 0 (reset to e_0)
  if (ti == 0) {
#pragma unroll
    for (int c = 0; c < 8; ++c) rowk[0][c0 + c] = a[0][c];
  }
  if (tj == 0) {
    if (ti == 0) pinv[0] = recip(a[0][0]);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      colk[0][r0 + r] = a[r][0] - T(r0 + r == 0 ? 1 : 0);
      a[r][0] = T(r0 + r == 0 ? 1 : 0);
    }
  }
  const int steps = (b + 7) & ~7;
  for (int g = 0; g < steps; g += 8) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int k = g + s, kn = k + 1;
      const int buf = s & 1, nb = buf ^ 1;  // k parity (g is a multiple of 8)
      __syncthreads();
      const T ip = pinv[buf];
      T u[8], v[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) u[r] = colk[buf][r0 + r];
#pragma unroll
      for (int c = 0; c < 8; ++c) v[c] = (c0 + c == k) ? ip : rowk[buf][c0 + c] * ip;
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c = 0; c < 8; ++c) a[r][c] = fma(-u[r], v[c], a[r][c]);
      // next pivot: register row / column sn of the thread row / column gn
      const int sn = (s + 1) & 7;
      const int gn = kn >> 3;
      if (kn < NB) {
        if (ti == gn) {
#pragma unroll
          for (int c = 0; c < 8; ++c) rowk[nb][c0 + c] = a[sn][c];
        }
        if (tj == gn) {
          // the owner of the next pivot publishes its reciprocal, so that no
          // thread divides between the barrier and its update
          if (ti == gn) pinv[nb] = recip(a[sn][sn]);
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            colk[nb][r0 + r] = a[r][sn] - T(r0 + r == kn ? 1 : 0);
            a[r][sn] = T(r0 + r == kn ? 1 : 0);
          }
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 8; ++r)
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int i = r0 + r, j = c0 + c;
      if (i < b && j < b) out[ROWMAJOR_OUT ? int64_t(i) * b + j : int64_t(j) * b + i] = a[r][c];
    }
}

void launch_gj_block_inverse(const double* X, int64_t ldx, double* out, int b, hipStream_t st) {
  hipLaunchKernelGGL((k_gj_block_inverse_t<double, false>), dim3(1), dim3(256), 0, st, X, ldx, out, b);
}

void launch_gj_block_inverse_f32(const float* X, int64_t ldx, float* out_rowmajor, int b, hipStream_t st) {
  hipLaunchKernelGGL((k_gj_block_inverse_t<float, true>), dim3(1), dim3(256), 0, st, X, ldx, out_rowmajor, b);
}

// FP32 take-columns with C row-major (n x b, C[i * b + j]).
__global__ void k_gj_take_columns_f32(float* X, int64_t n, int p0, int b, float* C) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= n * b) return;
  const int64_t i = q % n, j = q / n;
  float* x = X + (p0 + j) * n + i;
  const bool pr = (i >= p0 && i < p0 + b);
  C[i * b + j] = pr ? 0.0f : *x;
  *x = (pr && i - p0 == j) ? 1.0f : 0.0f;
}

void launch_gj_take_columns_f32(float* X, int64_t n, int p0, int b, float* C, hipStream_t st) {
  const int64_t m = n * b;
  hipLaunchKernelGGL(k_gj_take_columns_f32, dim3(unsigned((m + 255) / 256)), dim3(256), 0, st, X, n, p0, b, C);
}

// out (n2 x n2, FP32) = [[in, 0], [0, I]] for in n x n FP64 row-major
__global__ void k_embed_f32(const double* in, int n, float* out, int n2) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= int64_t(n2) * n2) return;
  const int64_t i = q / n2, j = q % n2;
  out[q] = (i < n && j < n) ? float(in[i * n + j]) : (i == j ? 1.0f : 0.0f);
}

void launch_embed_f32(const double* in, int n, float* out, int n2, hipStream_t st) {
  const int64_t m = int64_t(n2) * n2;
  hipLaunchKernelGGL(k_embed_f32, dim3(unsigned((m + 255) / 256)), dim3(256), 0, st, in, n, out, n2);
}

__global__ void k_transpose_f32(const float* in, float* out, int n) {
  __shared__ float tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const int i = by + k, j = bx + threadIdx.x;
    if (i < n && j < n) tile[k][threadIdx.x] = in[int64_t(i) * n + j];
  }
  __syncthreads();
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const int i = bx + k, j = by + threadIdx.x;
    if (i < n && j < n) out[int64_t(i) * n + j] = tile[threadIdx.x][k];
  }
}

void launch_transpose_f32(const float* in, float* out, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_transpose_f32, dim3((n + 31) / 32, (n + 31) / 32), dim3(32, 8), 0, st, in, out, n);
}

// Column block p0..p0+b of X (col-major, n x n): copy it to C (n x b) with the
// pivot rows zeroed, and overwrite it in X with the unit block.
__global__ void k_gj_take_columns(double* X, int64_t n, int p0, int b, double* C) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= n * b) return;
  const int64_t i = q % n, j = q / n;
  double* x = X + (p0 + j) * n + i;
  const bool pr = (i >= p0 && i < p0 + b);
  C[j * n + i] = pr ? 0.0 : *x;
  *x = (pr && i - p0 == j) ? 1.0 : 0.0;
}

void launch_gj_take_columns(double* X, int64_t n, int p0, int b, double* C, hipStream_t st) {
  const int64_t m = n * b;
  hipLaunchKernelGGL(k_gj_take_columns, dim3(unsigned((m + 255) / 256)), dim3(256), 0, st, X, n, p0, b, C);
}

// Dense complex vectors: y = alpha * M x for real dense M applied to the
// two trace components at once (one read of M for D and N and all vectors);
// one wavefront per 8 / NR rows, so that each x load serves several rows.
// Each lane loads 16 bytes of a row at a time (4 floats or 2 doubles; the
// leading dimension is a multiple of 4 and the padding columns are zero),
// non-temporal since the matrix is streamed once per application.
template <typename M, int NR, int KS>
__global__ __launch_bounds__(256) void k_gemv_real2(const M* __restrict__ Mat, int64_t ld, int rows, int cols,
                                                    double alpha, const double* __restrict__ x, double* y,
                                                    int64_t vstride, int64_t cstride) {
  constexpr int VEC = 16 / int(sizeof(M));
  constexpr int ROWS = NR >= 8 ? 1 : 8 / NR;
  typedef M Vt __attribute__((ext_vector_type(VEC)));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int part = wv % KS;
  const int row0 = ROWS * (blockIdx.x * (4 / KS) + wv / KS);
  const bool live = row0 < rows;  // no early exit: every wavefront reaches the barrier
  const Vt* mr[ROWS];
#pragma unroll
  for (int h = 0; h < ROWS; ++h) mr[h] = reinterpret_cast<const Vt*>(Mat + int64_t(min(row0 + h, rows - 1)) * ld);
  double a[ROWS][NR][4];
#pragma unroll
  for (int h = 0; h < ROWS; ++h)
#pragma unroll
    for (int r = 0; r < NR; ++r) a[h][r][0] = a[h][r][1] = a[h][r][2] = a[h][r][3] = 0.0;
  const int nq = (cols + VEC - 1) / VEC;
  const int q0 = int(int64_t(nq) * part / KS), q1 = live ? int(int64_t(nq) * (part + 1) / KS) : q0;
  for (int q = q0 + lane; q < q1; q += 64) {
    Vt m[ROWS];
#pragma unroll
    for (int h = 0; h < ROWS; ++h) m[h] = __builtin_nontemporal_load(&mr[h][q]);
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const int j = q * VEC + v;
        double2 x0 = {0.0, 0.0}, x1 = {0.0, 0.0};
        if (j < cols) {
          x0 = *reinterpret_cast<const double2*>(x + 2 * (int64_t(r) * vstride + j));
          x1 = *reinterpret_cast<const double2*>(x + 2 * (int64_t(r) * vstride + cstride + j));
        }
#pragma unroll
        for (int h = 0; h < ROWS; ++h) {
          const double mv = double(m[h][v]);
          a[h][r][0] += mv * x0.x;
          a[h][r][1] += mv * x0.y;
          a[h][r][2] += mv * x1.x;
          a[h][r][3] += mv * x1.y;
        }
      }
  }
#pragma unroll
  for (int h = 0; h < ROWS; ++h)
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) a[h][r][q] = wsum(a[h][r][q]);
  if (KS > 1) {
    __shared__ double red[4][ROWS * NR * 4];
    if (lane == 0 && part > 0) {
#pragma unroll
      for (int h = 0; h < ROWS; ++h)
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
          for (int q = 0; q < 4; ++q) red[wv][(h * NR + r) * 4 + q] = a[h][r][q];
    }
    __syncthreads();
    if (lane == 0 && part == 0) {
#pragma unroll
      for (int p = 1; p < KS; ++p)
#pragma unroll
        for (int h = 0; h < ROWS; ++h)
#pragma unroll
          for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int q = 0; q < 4; ++q) a[h][r][q] += red[wv + p][(h * NR + r) * 4 + q];
    }
  }
  if (lane == 0 && part == 0 && live) {
#pragma unroll
    for (int h = 0; h < ROWS; ++h) {
      if (row0 + h >= rows) break;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        double* q0p = y + 2 * (int64_t(r) * vstride + row0 + h);
        double* q1p = q0p + 2 * cstride;
        q0p[0] = alpha * a[h][r][0];
        q0p[1] = alpha * a[h][r][1];
        q1p[0] = alpha * a[h][r][2];
        q1p[1] = alpha * a[h][r][3];
      }
    }
  }
}

// Column split only for few row groups: on the 7680-column mass inverse the
// 2-way split is 1.4x slower than one wavefront per row group (more
// concurrent row streams), on 1920 / 3840 columns 4- / 2-way are ~10% faster.
template <typename M, int NR>
static void real2_launch(const M* Mat, int64_t ld, int rows, int cols, double alpha, const double* xx, double* yy,
                         int64_t vstride, int64_t cstride, hipStream_t st) {
  constexpr int ROWS = NR >= 8 ? 1 : 8 / NR;
  const int groups = (rows + ROWS - 1) / ROWS;
  const dim3 block(256);
  if (groups <= 256)
    hipLaunchKernelGGL((k_gemv_real2<M, NR, 4>), dim3(unsigned(groups)), block, 0, st, Mat, ld, rows, cols, alpha, xx,
                       yy, vstride, cstride);
  else if (groups <= 512)
    hipLaunchKernelGGL((k_gemv_real2<M, NR, 2>), dim3(unsigned((groups + 1) / 2)), block, 0, st, Mat, ld, rows, cols,
                       alpha, xx, yy, vstride, cstride);
  else
    hipLaunchKernelGGL((k_gemv_real2<M, NR, 1>), dim3(unsigned((groups + 3) / 4)), block, 0, st, Mat, ld, rows, cols,
                       alpha, xx, yy, vstride, cstride);
}

template <typename M>
void launch_gemv_real2(const M* Mat, int64_t ld, int rows, int cols, double alpha, const double* x, double* y,
                       int nrhs, int64_t vstride, int64_t cstride, hipStream_t st) {
  for (int r0 = 0; r0 < nrhs;) {
    const int left = nrhs - r0;
    const double* xx = x + 2 * int64_t(r0) * vstride;
    double* yy = y + 2 * int64_t(r0) * vstride;
    if (left >= 4) {
      real2_launch<M, 4>(Mat, ld, rows, cols, alpha, xx, yy, vstride, cstride, st);
      r0 += 4;
    } else {
      real2_launch<M, 1>(Mat, ld, rows, cols, alpha, xx, yy, vstride, cstride, st);
      r0 += 1;
    }
  }
}
template void launch_gemv_real2<double>(const double*, int64_t, int, int, double, const double*, double*, int,
                                        int64_t, int64_t, hipStream_t);
template void launch_gemv_real2<float>(const float*, int64_t, int, int, double, const double*, double*, int, int64_t,
                                       int64_t, hipStream_t);

// ---------------------------------------------------------------------------
// Truncated sparse copy of an FP32 inverse mass matrix (mixed-precision P).
// The inverse of the well-conditioned mixed mass matrix decays with the
// graph distance between functions; entries below 2^-27 of their row's
// largest lie under the FP32 rounding of the stored inverse and are dropped
// (on the 7680-edge sphere: 584 of 7680 per row kept, product error 5e-8
// against 3e-8 for the dense FP32 copy).  One wavefront per row.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_trunc_count(const T* __restrict__ A, int64_t ld, int rows, int cols, T rel,
                                                     int32_t* cnt, T* thr) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const T* a = A + int64_t(row) * ld;
  T mx = T(0);
  for (int j = lane; j < cols; j += 64) mx = fmax(mx, fabs(a[j]));
  for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  const T t = rel * mx;
  int c = 0;
  for (int j = lane; j < cols; j += 64) c += (fabs(a[j]) >= t && a[j] != T(0)) ? 1 : 0;
  for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
  if (lane == 0) {
    cnt[row] = c;
    thr[row] = t;
  }
}

// rowptr[0] = 0, rowptr[i + 1] = cnt[0] + ... + cnt[i]: one workgroup, each
// thread sums a contiguous run of rows, then the run totals are scanned in
// order by one thread
__global__ __launch_bounds__(1024) void k_scan_counts(const int32_t* cnt, int rows, int64_t* rowptr) {
  __shared__ int64_t tot[1024];
  const int t = threadIdx.x;
  const int per = (rows + 1023) / 1024;
  const int r0 = min(rows, t * per), r1 = min(rows, r0 + per);
  int64_t s = 0;
  for (int r = r0; r < r1; ++r) s += cnt[r];
  tot[t] = s;
  __syncthreads();
  if (t == 0) {
    int64_t run = 0;
    for (int q = 0; q < 1024; ++q) {
      const int64_t v = tot[q];
      tot[q] = run;
      run += v;
    }
    rowptr[0] = 0;
  }
  __syncthreads();
  int64_t run = tot[t];
  for (int r = r0; r < r1; ++r) {
    run += cnt[r];
    rowptr[r + 1] = run;
  }
}

// kept entries of each row in ascending column order (wavefront ballot)
template <typename T>
__global__ __launch_bounds__(256) void k_trunc_fill(const T* __restrict__ A, int64_t ld, int rows, int cols,
                                                    const T* thr, const int64_t* rowptr, int32_t* col, T* val) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const T* a = A + int64_t(row) * ld;
  const T t = thr[row];
  int64_t base = rowptr[row];
  const uint64_t below = (uint64_t(1) << lane) - 1;
  for (int j0 = 0; j0 < cols; j0 += 64) {
    const int j = j0 + lane;
    const T v = j < cols ? a[j] : T(0);
    const bool keep = j < cols && fabs(v) >= t && v != T(0);
    const uint64_t m = __ballot(keep);
    if (keep) {
      const int64_t pos = base + __popcll(m & below);
      col[pos] = j;
      val[pos] = v;
    }
    base += __popcll(m);
  }
}

template <typename T>
void build_truncated_inverse(const T* A, int64_t ld, int n, T rel, int32_t* cnt, T* thr, int64_t* rowptr,
                             hipStream_t st) {
  hipLaunchKernelGGL((k_trunc_count<T>), dim3(unsigned((n + 3) / 4)), dim3(256), 0, st, A, ld, n, n, rel, cnt, thr);
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, st, cnt, n, rowptr);
}
template void build_truncated_inverse<float>(const float*, int64_t, int, float, int32_t*, float*, int64_t*,
                                             hipStream_t);
template void build_truncated_inverse<double>(const double*, int64_t, int, double, int32_t*, double*, int64_t*,
                                              hipStream_t);

template <typename T>
void fill_truncated_inverse(const T* A, int64_t ld, int n, const T* thr, const int64_t* rowptr, int32_t* col, T* val,
                            hipStream_t st) {
  hipLaunchKernelGGL((k_trunc_fill<T>), dim3(unsigned((n + 3) / 4)), dim3(256), 0, st, A, ld, n, n, thr, rowptr, col,
                     val);
}
template void fill_truncated_inverse<float>(const float*, int64_t, int, const float*, const int64_t*, int32_t*,
                                            float*, hipStream_t);
template void fill_truncated_inverse<double>(const double*, int64_t, int, const double*, const int64_t*, int32_t*,
                                             double*, hipStream_t);

// ---------------------------------------------------------------------------
// Inverse of the mixed mass matrix by a Chebyshev iteration from the right,
//   R_k = I - X_k M,  D_k = rho_k rho_{k-1} D_{k-1} + (2 rho_k / c) R_k,
//   X_{k+1} = X_k + D_k,  rho_k = 1 / (2 sigma - rho_{k-1}),
// for a spectrum inside [d - c, d + c] (sigma = d / c), starting from
// X_1 = D_0 = I / d.  Row i of the iteration involves row i of X only, so a
// workgroup keeps RB rows of X in LDS and forms (X M)_ij for every column j
// from the CSC of the sparse M (about 19 entries per column), accumulating in
// FP64.  Each launch is one step over all rows; it also leaves the partial
// sums of ||R_k||_F^2 per workgroup.  first: X_1 and D_0 are generated.
// ---------------------------------------------------------------------------
template <typename T, int RB>
struct RowPack {
  T v[RB];
};

template <typename T, int RB, int W>
__global__ __launch_bounds__(512) void k_cheb_step(T* X, T* D, int64_t ld, int n, const int32_t* __restrict__ eidx,
                                                    const T* __restrict__ eval, double cD, double cR, double inv_d,
                                                    int first, double* rn_part) {
  extern __shared__ __align__(16) unsigned char cheb_raw[];
  // rows interleaved: xs[k] holds X[row0 + r][k] for the RB rows, one vector read per entry of M
  RowPack<T, RB>* xs = reinterpret_cast<RowPack<T, RB>*>(cheb_raw);
  __shared__ double red[512];
  const int row0 = blockIdx.x * RB;
  const int nr = min(RB, n - row0);
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    RowPack<T, RB> pk;
#pragma unroll
    for (int r = 0; r < RB; ++r)
      pk.v[r] = r >= nr ? T(0) : (first ? T(j == row0 + r ? inv_d : 0.0) : X[int64_t(row0 + r) * ld + j]);
    xs[j] = pk;
  }
  __syncthreads();
  double ss = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    // column j of M, W slots (zero-padded), entry-major: coalesced over j
    int kk[W];
    T vv[W];
#pragma unroll
    for (int q = 0; q < W; ++q) {
      kk[q] = eidx[int64_t(q) * n + j];
      vv[q] = eval[int64_t(q) * n + j];
    }
    double t[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) t[r] = 0.0;
#pragma unroll
    for (int q = 0; q < W; ++q) {
      const RowPack<T, RB> xk = xs[kk[q]];
#pragma unroll
      for (int r = 0; r < RB; ++r) t[r] += double(xk.v[r]) * double(vv[q]);
    }
    const RowPack<T, RB> xj = xs[j];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      if (r >= nr) break;
      const int i = row0 + r;
      const int64_t o = int64_t(i) * ld + j;
      const double Rv = (j == i ? 1.0 : 0.0) - t[r];
      const double dprev = first ? (j == i ? inv_d : 0.0) : double(D[o]);
      const double dn = cD * dprev + cR * Rv;
      D[o] = T(dn);
      X[o] = T(double(xj.v[r]) + dn);
      ss += Rv * Rv;
    }
  }
  red[threadIdx.x] = ss;
  __syncthreads();
  for (int q = blockDim.x / 2; q > 0; q >>= 1) {
    if (threadIdx.x < q) red[threadIdx.x] += red[threadIdx.x + q];
    __syncthreads();
  }
  if (threadIdx.x == 0) rn_part[blockIdx.x] = red[0];
}

// ELL copy (W slots per column, entry-major, padding: index j, value 0) of
// the CSC colptr / rowidx / val
template <typename T>
__global__ void k_csc_to_ell(const int64_t* colptr, const int32_t* rowidx, const double* val, int n, int W,
                             int32_t* eidx, T* eval) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t p0 = colptr[j];
  const int c = int(colptr[j + 1] - p0);
  for (int q = 0; q < W; ++q) {
    eidx[int64_t(q) * n + j] = q < c ? rowidx[p0 + q] : j;
    eval[int64_t(q) * n + j] = q < c ? T(val[p0 + q]) : T(0);
  }
}
template <typename T>
void launch_csc_to_ell(const int64_t* colptr, const int32_t* rowidx, const double* val, int n, int W, int32_t* eidx,
                       T* eval, hipStream_t st) {
  hipLaunchKernelGGL((k_csc_to_ell<T>), dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, colptr, rowidx, val, n, W,
                     eidx, eval);
}
template void launch_csc_to_ell<float>(const int64_t*, const int32_t*, const double*, int, int, int32_t*, float*,
                                       hipStream_t);

// rows per workgroup: 2 when two rows of X fit in 136 KB of LDS, else 1
// (0: a row does not fit).  Measured on the 7680-edge sphere, whole inverse:
// 4 rows (one workgroup per CU) 8.6 ms, 2 rows (two per CU, their load and
// gather phases overlap) 7.2 ms, 1 row (the ELL copy of M_A re-read by twice
// as many workgroups) 9.7 ms.
template <typename T>
int cheb_rows(int n) {
  const int64_t per = int64_t(n) * sizeof(T);
  const int rb = int(std::min<int64_t>(2, (136 * 1024) / std::max<int64_t>(per, 1)));
  return rb >= 2 ? 2 : rb;
}
template int cheb_rows<float>(int);

template <typename T, int RB, int W>
static void cheb_launch(T* X, T* D, int64_t ld, int n, const int32_t* eidx, const T* eval, double cD, double cR,
                        double inv_d, bool first, double* rn_part, hipStream_t st) {
  static bool attr = false;  // beyond the default dynamic LDS limit
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cheb_step<T, RB, W>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 136 * 1024);
    attr = true;
  }
  const dim3 grid(unsigned((n + RB - 1) / RB)), block(512);
  hipLaunchKernelGGL((k_cheb_step<T, RB, W>), grid, block, size_t(RB) * n * sizeof(T), st, X, D, ld, n, eidx, eval, cD,
                     cR, inv_d, int(first), rn_part);
}

template <typename T, int W>
static void cheb_launch_rb(T* X, T* D, int64_t ld, int n, const int32_t* eidx, const T* eval, double cD, double cR,
                           double inv_d, bool first, double* rn_part, hipStream_t st) {
  const int rb = cheb_rows<T>(n);
  if (rb == 2)
    cheb_launch<T, 2, W>(X, D, ld, n, eidx, eval, cD, cR, inv_d, first, rn_part, st);
  else
    cheb_launch<T, 1, W>(X, D, ld, n, eidx, eval, cD, cR, inv_d, first, rn_part, st);
}

int cheb_width(int maxcount) {
  for (int w : {16, 24, 32, 48, 64})
    if (maxcount <= w) return w;
  return 0;
}

template <typename T>
void launch_cheb_step(T* X, T* D, int64_t ld, int n, const int32_t* eidx, const T* eval, int W, double cD, double cR,
                      double inv_d, bool first, double* rn_part, hipStream_t st) {
  switch (W) {
    case 16: cheb_launch_rb<T, 16>(X, D, ld, n, eidx, eval, cD, cR, inv_d, first, rn_part, st); break;
    case 24: cheb_launch_rb<T, 24>(X, D, ld, n, eidx, eval, cD, cR, inv_d, first, rn_part, st); break;
    case 32: cheb_launch_rb<T, 32>(X, D, ld, n, eidx, eval, cD, cR, inv_d, first, rn_part, st); break;
    case 48: cheb_launch_rb<T, 48>(X, D, ld, n, eidx, eval, cD, cR, inv_d, first, rn_part, st); break;
    default: cheb_launch_rb<T, 64>(X, D, ld, n, eidx, eval, cD, cR, inv_d, first, rn_part, st); break;
  }
}
template void launch_cheb_step<float>(float*, float*, int64_t, int, const int32_t*, const float*, int, double, double,
                                      double, bool, double*, hipStream_t);

// X[i][i] = 1 for the padding rows n <= i < ld (the inverse of [[M, 0], [0, I]])
template <typename T>
__global__ void k_identity_tail(T* X, int64_t ld, int n) {
  const int64_t i = n + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < ld) X[i * ld + i] = T(1);
}
template <typename T>
void launch_identity_tail(T* X, int64_t ld, int n, hipStream_t st) {
  if (ld > n) hipLaunchKernelGGL((k_identity_tail<T>), dim3(unsigned((ld - n + 255) / 256)), dim3(256), 0, st, X, ld, n);
}
template void launch_identity_tail<float>(float*, int64_t, int, hipStream_t);


// y = alpha * M x (M real CSR) on the two trace components of NR complex
// vectors: the same product as k_gemv_real2 from the truncated inverse.  One
// wavefront per row, lanes over the row's entries.
template <int NR, typename VT>
__global__ __launch_bounds__(256) void k_spmv_real2_csr(const int64_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col,
                                                        const VT* __restrict__ val, int rows, double alpha,
                                                        const double* __restrict__ x, double* y, int64_t vstride,
                                                        int64_t cstride, double beta) {
  // right-hand sides NR blockIdx.y .. NR blockIdx.y + NR - 1
  x += 2 * int64_t(blockIdx.y) * NR * vstride;
  y += 2 * int64_t(blockIdx.y) * NR * vstride;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  double acc[NR][4];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r][0] = acc[r][1] = acc[r][2] = acc[r][3] = 0.0;
  const int64_t p1 = rowptr[row + 1];
  // unrolled so that the index and value loads of later entries are in
  // flight while earlier ones gather x (the sum per lane stays in order)
#pragma unroll 4
  for (int64_t p = rowptr[row] + lane; p < p1; p += 64) {
    const int c = col[p];
    const double v = double(val[p]);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double2 x0 = *reinterpret_cast<const double2*>(x + 2 * (int64_t(r) * vstride + c));
      const double2 x1 = *reinterpret_cast<const double2*>(x + 2 * (int64_t(r) * vstride + cstride + c));
      acc[r][0] += v * x0.x;
      acc[r][1] += v * x0.y;
      acc[r][2] += v * x1.x;
      acc[r][3] += v * x1.y;
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[r][q] = wsum(acc[r][q]);
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      double* q0 = y + 2 * (int64_t(r) * vstride + row);
      double* q1 = q0 + 2 * cstride;
      if (beta == 0.0) {
        q0[0] = alpha * acc[r][0];
        q0[1] = alpha * acc[r][1];
        q1[0] = alpha * acc[r][2];
        q1[1] = alpha * acc[r][3];
      } else {
        q0[0] = alpha * acc[r][0] + beta * q0[0];
        q0[1] = alpha * acc[r][1] + beta * q0[1];
        q1[0] = alpha * acc[r][2] + beta * q1[0];
        q1[1] = alpha * acc[r][3] + beta * q1[1];
      }
    }
  }
}

template <typename VT>
static void spmv_real2_csr(const int64_t* rowptr, const int32_t* col, const VT* val, int rows, double alpha,
                           const double* x, double* y, int nrhs, int64_t vstride, int64_t cstride, hipStream_t st,
                           double beta) {
  // groups of 4 right-hand sides in one launch (grid.y over the groups), the
  // remainder one at a time in a second launch
  const unsigned gx = unsigned((rows + 3) / 4);
  const int n4 = nrhs / 4, r0 = 4 * n4;
  if (n4 > 0)
    hipLaunchKernelGGL((k_spmv_real2_csr<4, VT>), dim3(gx, unsigned(n4)), dim3(256), 0, st, rowptr, col, val, rows,
                       alpha, x, y, vstride, cstride, beta);
  if (nrhs > r0) {
    const int64_t o = 2 * int64_t(r0) * vstride;
    hipLaunchKernelGGL((k_spmv_real2_csr<1, VT>), dim3(gx, unsigned(nrhs - r0)), dim3(256), 0, st, rowptr, col, val,
                       rows, alpha, x + o, y + o, vstride, cstride, beta);
  }
}
// xt[(c nrhs + r) 4 + q] = (xD re, xD im, xN re, xN im)[q] of rhs r at column
// c; thread per (rhs, column), consecutive threads along the columns
__global__ void k_gather_cols(const double* __restrict__ x, int64_t vstride, int64_t cstride, int cols, int nrhs,
                              double* __restrict__ xt) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(cols) * nrhs) return;
  const int r = int(t / cols), c = int(t - int64_t(r) * cols);
  const double* xr = x + 2 * int64_t(r) * vstride;
  const double2 d = *reinterpret_cast<const double2*>(xr + 2 * int64_t(c));
  const double2 n = *reinterpret_cast<const double2*>(xr + 2 * (cstride + c));
  double* o = xt + (int64_t(c) * nrhs + r) * 4;
  *reinterpret_cast<double2*>(o) = d;
  *reinterpret_cast<double2*>(o + 2) = n;
}

// y = alpha M x (beta = 0) for every right-hand side, reading x from the
// gathered copy xt.  16 lanes per row (four rows per wavefront: the rows of
// M_A hold about 20 entries), each wavefront's rows taking every group of 4
// right-hand sides in turn (the remainder as a last, partial group): one
// wavefront per 4 rows for the whole batch instead of one per row and group.
// Per group: lane sums over its entries in order, then over the 16 lanes.
__global__ __launch_bounds__(256) void k_spmv_real2_csr_t(const int64_t* __restrict__ rowptr,
                                                          const int32_t* __restrict__ col,
                                                          const double* __restrict__ val, int rows, double alpha,
                                                          const double* __restrict__ xt, int nrhs, double* y,
                                                          int64_t vstride, int64_t cstride) {
  const int lane = threadIdx.x & 63, l16 = lane & 15;
  const int row = blockIdx.x * 16 + (threadIdx.x >> 4);
  const bool live = row < rows;  // every lane takes part in the row sums
  const int64_t p0 = live ? rowptr[row] : 0, p1 = live ? rowptr[row + 1] : 0;
  for (int rb = 0; rb < nrhs; rb += 4) {
    const int nr = min(4, nrhs - rb);
    double acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r][0] = acc[r][1] = acc[r][2] = acc[r][3] = 0.0;
    for (int64_t p = p0 + l16; p < p1; p += 16) {
      const int c = col[p];
      const double v = val[p];
      const double2* src = reinterpret_cast<const double2*>(xt + (int64_t(c) * nrhs + rb) * 4);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (r < nr) {
          const double2 x0 = src[2 * r], x1 = src[2 * r + 1];
          acc[r][0] += v * x0.x;
          acc[r][1] += v * x0.y;
          acc[r][2] += v * x1.x;
          acc[r][3] += v * x1.y;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[r][q] = row_sum<16>(acc[r][q]);
    if (live && l16 == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (r < nr) {
          double* q0 = y + 2 * (int64_t(rb + r) * vstride + row);
          double* q1 = q0 + 2 * cstride;
          q0[0] = alpha * acc[r][0];
          q0[1] = alpha * acc[r][1];
          q1[0] = alpha * acc[r][2];
          q1[1] = alpha * acc[r][3];
        }
      }
    }
  }
}

void launch_spmv_real2_csr_t(const int64_t* rowptr, const int32_t* col, const double* val, int rows, int cols,
                             double alpha, const double* x, double* y, int nrhs, int64_t vstride, int64_t cstride,
                             double* xt, hipStream_t st) {
  const int64_t n = int64_t(cols) * nrhs;
  hipLaunchKernelGGL(k_gather_cols, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, x, vstride, cstride, cols, nrhs,
                     xt);
  hipLaunchKernelGGL(k_spmv_real2_csr_t, dim3(unsigned((rows + 15) / 16)), dim3(256), 0, st, rowptr, col, val, rows,
                     alpha, xt, nrhs, y, vstride, cstride);
}

void launch_spmv_real2_csr(const int64_t* rowptr, const int32_t* col, const float* val, int rows, double alpha,
                           const double* x, double* y, int nrhs, int64_t vstride, int64_t cstride, hipStream_t st,
                           double beta) {
  spmv_real2_csr(rowptr, col, val, rows, alpha, x, y, nrhs, vstride, cstride, st, beta);
}
void launch_spmv_real2_csr(const int64_t* rowptr, const int32_t* col, const double* val, int rows, double alpha,
                           const double* x, double* y, int nrhs, int64_t vstride, int64_t cstride, hipStream_t st,
                           double beta) {
  spmv_real2_csr(rowptr, col, val, rows, alpha, x, y, nrhs, vstride, cstride, st, beta);
}

// sum of v over the 1024 threads of the workgroup, the same in every thread:
// each wavefront's sum (DPP within rows of 16, then across rows), then the 16
// wavefront sums in order.  The two slot sets red[0], red[1] alternate
// between consecutive calls (set): a wavefront writes a set only after every
// wavefront has passed the previous call's barrier, so after every read of
// that set in the call before.  One barrier per call.
__device__ __forceinline__ double block_sum1024(double v, double (*red)[16], int& set) {
  v = row_sum<32>(v);
  v += __shfl_xor(v, 32, WAVE);
  if ((threadIdx.x & 63) == 0) red[set][threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < 16; ++w) t += red[set][w];
  set ^= 1;
  return t;
}

// Conjugate gradients for G x = b with G real symmetric positive definite
// (CSR; rowptr of this block, col and val global) and complex b, one
// workgroup of 1024 threads per right-hand side, from x = 0 until
// |r|^2 <= tol2 |b|^2 or maxit steps.  Each thread takes every 1024-th
// element; the sums go through block_sum1024, so the iterates do not depend
// on timing.  work: r, p, q (2n doubles each) per right-hand side.
__global__ __launch_bounds__(1024) void k_gram_cg(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                                  const double* __restrict__ val, int n, const double* b,
                                                  int64_t bstride, double* x, int64_t xstride, double* work,
                                                  double tol2, int maxit) {
  __shared__ double red[2][16];
  int set = 0;
  const int v = blockIdx.x;
  const double* bv = b + 2 * int64_t(v) * bstride;
  double* xv = x + 2 * int64_t(v) * xstride;
  double* r = work + 6 * int64_t(v) * n;
  double* p = r + 2 * int64_t(n);
  double* q = p + 2 * int64_t(n);
  double sum = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) {
    const double br = bv[2 * i], bi = bv[2 * i + 1];
    xv[2 * i] = 0.0;
    xv[2 * i + 1] = 0.0;
    r[2 * i] = br;
    r[2 * i + 1] = bi;
    p[2 * i] = br;
    p[2 * i + 1] = bi;
    sum += br * br + bi * bi;
  }
  double rr = block_sum1024(sum, red, set);  // its barrier also publishes r and p to the workgroup
  const double rr0 = rr;
  for (int it = 0; it < maxit && rr > tol2 * rr0; ++it) {  // rr is the same in every thread
    sum = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) {
      double qr = 0.0, qi = 0.0;
      for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        const double g = val[k];
        const int j = col[k];
        qr += g * p[2 * j];
        qi += g * p[2 * j + 1];
      }
      q[2 * i] = qr;
      q[2 * i + 1] = qi;
      sum += p[2 * i] * qr + p[2 * i + 1] * qi;
    }
    const double pq = block_sum1024(sum, red, set);
    const double al = pq > 0 ? rr / pq : 0.0;
    sum = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) {
      xv[2 * i] += al * p[2 * i];
      xv[2 * i + 1] += al * p[2 * i + 1];
      const double rr_ = r[2 * i] - al * q[2 * i], ri_ = r[2 * i + 1] - al * q[2 * i + 1];
      r[2 * i] = rr_;
      r[2 * i + 1] = ri_;
      sum += rr_ * rr_ + ri_ * ri_;
    }
    const double rn = block_sum1024(sum, red, set);
    const double be = rr > 0 ? rn / rr : 0.0;
    rr = rn;
    for (int i = threadIdx.x; i < n; i += 1024) {
      p[2 * i] = r[2 * i] + be * p[2 * i];
      p[2 * i + 1] = r[2 * i + 1] + be * p[2 * i + 1];
    }
    __syncthreads();  // p complete before the next product reads it
  }
}

void launch_gram_cg(const int64_t* rowptr, const int32_t* col, const double* val, int n, const double* b,
                    int64_t bstride, double* x, int64_t xstride, int nvec, double* work, double tol2, int maxit,
                    hipStream_t st) {
  if (n <= 0 || nvec <= 0) return;
  hipLaunchKernelGGL(k_gram_cg, dim3(unsigned(nvec)), dim3(1024), 0, st, rowptr, col, val, n, b, bstride, x, xstride,
                     work, tol2, maxit);
}

// out[i * ldo + j] = in[i * n + j] (j < n), 0 for n <= j < ldo
template <typename T>
__global__ void k_repack(const double* in, int n, T* out, int64_t ldo) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= int64_t(n) * ldo) return;
  const int64_t i = q / ldo, j = q % ldo;
  out[q] = j < n ? T(in[i * n + j]) : T(0);
}

template <typename T>
void launch_repack(const double* in, int n, T* out, int64_t ldo, hipStream_t st) {
  const int64_t m = int64_t(n) * ldo;
  hipLaunchKernelGGL((k_repack<T>), dim3(unsigned((m + 255) / 256)), dim3(256), 0, st, in, n, out, ldo);
}
template void launch_repack<double>(const double*, int, double*, int64_t, hipStream_t);
template void launch_repack<float>(const double*, int, float*, int64_t, hipStream_t);

}  // namespace pmchwt


