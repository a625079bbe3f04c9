// Sparse approximate inverse of the mixed mass matrix M_A (Section 3.2; the
// preconditioner applies M_A^-1 and M_P^-1 = -M_A^-T).  The entries of M_A^-1
// decay geometrically with the graph distance between functions (about a
// factor 5 per step of M_A's sparsity graph on the meshes measured), so row i
// of the inverse is computed only on the ball of columns reachable from i in
// L steps of that graph, by the Chebyshev iteration from the right
//   R_k = I - X_k M,  D_k = rho_k rho_{k-1} D_{k-1} + (2 rho_k / c) R_k,
//   X_{k+1} = X_k + D_k,  X_1 = D_0 = I / d,
// for a spectrum inside [d - c, d + c].  Row i of the iteration involves row i
// of X only, and X_k = p_k(M) is supported in the k-step ball, so restricting
// the row to the L-ball drops only entries below the decay at distance L.
//
// Pass 1 (one workgroup per row, small LDS, many rows per CU): breadth-first
// search over M's rows into an LDS hash table, then a bitonic sort of the
// ball's columns, written to a padded per-row buffer with the ball's size.
// Pass 2 (one workgroup per row, one ball column per thread): the thread of
// column q keeps the local positions and values of column q of M (at most
// SPINV_W entries) in registers, so every Chebyshev step is a gather of X_k
// from LDS in a fixed order: deterministic, with no global reads inside the
// iteration.  Values are written as a CSR row in column order.
#include "common.hpp"
#include "kernels.hpp"

namespace pmchwt {

constexpr int SPINV_BALL_THREADS = 256;
constexpr int SPINV_CAP = 1024;   // columns per row at most; also the pass-2 workgroup size
constexpr int SPINV_HASH = 2048;  // hash slots (power of two, >= 2 SPINV_CAP)
constexpr int SPINV_W = 24;       // entries per column of M at most (M_A has 19 on regular meshes)

__device__ __forceinline__ uint32_t spinv_hash(int32_t j) { return (uint32_t(j) * 2654435761u >> 7) & (SPINV_HASH - 1); }

// insert j; returns false if the ball is full (the row is refused)
__device__ __forceinline__ void spinv_insert(int32_t* keys, int32_t* cols, int* s_cnt, int* s_over, int32_t j) {
  if (*(volatile int*)s_cnt >= SPINV_CAP) {
    *s_over = 1;
    return;
  }
  uint32_t slot = spinv_hash(j);
  for (int probe = 0; probe < SPINV_HASH; ++probe) {
    const int32_t prev = atomicCAS(&keys[slot], -1, j);
    if (prev == -1) {
      const int idx = atomicAdd(s_cnt, 1);
      if (idx < SPINV_CAP)
        cols[idx] = j;
      else
        *s_over = 1;
      return;
    }
    if (prev == j) return;
    slot = (slot + 1) & (SPINV_HASH - 1);
  }
  *s_over = 1;
}

__global__ __launch_bounds__(SPINV_BALL_THREADS) void k_spinv_ball(SpInvJob J) {
  __shared__ int32_t keys[SPINV_HASH];
  __shared__ int32_t cols[SPINV_CAP];
  __shared__ int s_cnt, s_over;
  for (int i = blockIdx.x; i < J.n; i += gridDim.x) {
    for (int s = threadIdx.x; s < SPINV_HASH; s += SPINV_BALL_THREADS) keys[s] = -1;
    if (threadIdx.x == 0) {
      s_cnt = 0;
      s_over = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) spinv_insert(keys, cols, &s_cnt, &s_over, i);
    __syncthreads();
    int lo = 0, hi = 1;
    bool over = false;
    for (int lv = 0; lv < J.hops && !over; ++lv) {
      for (int p = lo + threadIdx.x; p < hi; p += SPINV_BALL_THREADS) {
        const int jp = cols[p];
        for (int64_t e = J.rp[jp]; e < J.rp[jp + 1]; ++e) spinv_insert(keys, cols, &s_cnt, &s_over, J.ci[e]);
      }
      __syncthreads();
      lo = hi;
      hi = min(s_cnt, SPINV_CAP);
      over = s_over != 0;
      __syncthreads();
    }
    if (over) {
      if (threadIdx.x == 0) J.count[i] = -1;
      __syncthreads();
      continue;
    }
    const int B = hi;
    // bitonic sort of the ball's columns, padded with INT_MAX to a power of two
    int P = 1;
    while (P < B) P <<= 1;
    for (int p = B + threadIdx.x; p < P; p += SPINV_BALL_THREADS) cols[p] = 0x7fffffff;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1)
      for (int jj = k >> 1; jj > 0; jj >>= 1) {
        for (int t = threadIdx.x; t < P; t += SPINV_BALL_THREADS) {
          const int u = t ^ jj;
          if (u > t) {
            const int32_t a = cols[t], b = cols[u];
            if ((a > b) == ((t & k) == 0)) {
              cols[t] = b;
              cols[u] = a;
            }
          }
        }
        __syncthreads();
      }
    int32_t* out = J.ball + int64_t(i) * SPINV_CAP;
    for (int q = threadIdx.x; q < B; q += SPINV_BALL_THREADS) out[q] = cols[q];
    if (threadIdx.x == 0) J.count[i] = B;
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(SPINV_CAP) void k_spinv_vals(SpInvJob J) {
  __shared__ int32_t keys[SPINV_HASH];
  __shared__ int16_t pos[SPINV_HASH];
  __shared__ double xs[SPINV_CAP], ds[SPINV_CAP];
  __shared__ double s_red[SPINV_CAP / WAVE];
  T* oval = static_cast<T*>(J.oval);
  const int q = threadIdx.x;
  const double dd = 0.5 * (J.a + J.b), cc = 0.5 * (J.b - J.a), sigma = dd / cc;
  for (int i = blockIdx.x; i < J.n; i += gridDim.x) {
    const int B = J.count[i];
    const int32_t* ball = J.ball + int64_t(i) * SPINV_CAP;
    for (int s = threadIdx.x; s < SPINV_HASH; s += SPINV_CAP) keys[s] = -1;
    __syncthreads();
    const bool live = q < B;
    const int32_t jq = live ? ball[q] : -1;
    if (live) {  // distinct keys: a free slot is found for each
      uint32_t slot = spinv_hash(jq);
      for (int probe = 0; probe < SPINV_HASH; ++probe) {
        if (atomicCAS(&keys[slot], -1, jq) == -1) {
          pos[slot] = int16_t(q);
          break;
        }
        slot = (slot + 1) & (SPINV_HASH - 1);
      }
    }
    __syncthreads();
    // column jq of M restricted to the ball, in M's column order
    int16_t lp[SPINV_W];
    float lv[SPINV_W];
    int len = 0;
    if (live) {
      const int64_t c0 = J.cp[jq];
      len = int(J.cp[jq + 1] - c0);
#pragma unroll
      for (int t = 0; t < SPINV_W; ++t) {
        lp[t] = -1;
        lv[t] = 0.0f;
        if (t < len) {
          const int32_t p = J.ri[c0 + t];
          uint32_t slot = spinv_hash(p);
          for (int probe = 0; probe < SPINV_HASH; ++probe) {
            const int32_t k = keys[slot];
            if (k == p) {
              lp[t] = pos[slot];
              break;
            }
            if (k == -1) break;
            slot = (slot + 1) & (SPINV_HASH - 1);
          }
          lv[t] = float(J.cv[c0 + t]);
        }
      }
      const double v0 = jq == i ? 1.0 / dd : 0.0;  // X_1 = D_0 = I / d
      xs[q] = v0;
      ds[q] = v0;
    }
    __syncthreads();
    double rho_prev = 1.0 / sigma, R = 0.0;
    for (int k = 1; k <= J.steps; ++k) {
      const double rho = 1.0 / (2.0 * sigma - rho_prev);
      if (live) {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < SPINV_W; ++t)
          if (lp[t] >= 0) s += xs[lp[t]] * double(lv[t]);
        R = (jq == i ? 1.0 : 0.0) - s;
      }
      __syncthreads();
      if (live) {
        const double dn = rho * rho_prev * ds[q] + (2.0 * rho / cc) * R;
        ds[q] = dn;
        xs[q] += dn;
      }
      __syncthreads();
      rho_prev = rho;
    }
    // the last step's residual over the ball, fixed-order sum
    double rs = live ? R * R : 0.0;
    for (int o = 32; o >= 1; o >>= 1) rs += __shfl_xor(rs, o, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0) s_red[threadIdx.x / WAVE] = rs;
    if (live) {
      const int64_t o = J.orp[i] + q;
      J.ocol[o] = jq;
      oval[o] = T(xs[q]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < SPINV_CAP / WAVE; ++w) t += s_red[w];
      J.res[i] = sqrt(t);
    }
    __syncthreads();
  }
}

// dense row-major copy (leading dimension ld, zeroed beforehand) of a CSR matrix
template <typename T>
__global__ __launch_bounds__(256) void k_csr_scatter(const int64_t* rowptr, const int32_t* col, const T* val, T* out,
                                                     int64_t ld) {
  const int i = blockIdx.x;
  for (int64_t e = rowptr[i] + threadIdx.x; e < rowptr[i + 1]; e += 256) out[int64_t(i) * ld + col[e]] = val[e];
}

void launch_csr_scatter_f32(const int64_t* rowptr, const int32_t* col, const float* val, int n, float* out, int64_t ld,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_csr_scatter<float>, dim3(unsigned(n)), dim3(256), 0, st, rowptr, col, val, out, ld);
}

// ---------------------------------------------------------------------------
// Transpose of an FP32 CSR matrix (the sparse M_A^-T from M_A^-1): column
// counts, a scan, records (row << 32 | entry) placed per column, sorted per
// column in LDS (k_sym_sort) so that the order is the row order whatever the
// order of the atomic placements, then the gather of columns and values.
// ---------------------------------------------------------------------------
__global__ void k_csr_colcount(const int32_t* __restrict__ col, int64_t nnz, int32_t* __restrict__ cnt) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < nnz) atomicAdd(&cnt[col[p]], 1);
}

__global__ void k_csr_tplace(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col, int n,
                             const int64_t* __restrict__ trowptr, int32_t* __restrict__ cur,
                             int64_t* __restrict__ rec) {
  const int i = blockIdx.x;
  if (i >= n) return;
  for (int64_t p = rowptr[i] + threadIdx.x; p < rowptr[i + 1]; p += blockDim.x) {
    const int j = col[p];
    rec[trowptr[j] + atomicAdd(&cur[j], 1)] = (int64_t(i) << 32) | int64_t(uint32_t(p));
  }
}

__global__ void k_csr_tgather(const int64_t* __restrict__ rec, int64_t nnz, const float* __restrict__ val,
                              int32_t* __restrict__ tcol, float* __restrict__ tval) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= nnz) return;
  const int64_t r = rec[q];
  tcol[q] = int32_t(r >> 32);
  tval[q] = val[uint32_t(r & 0xffffffffll)];
}

void launch_csr_colcount(const int32_t* col, int64_t nnz, int32_t* cnt, hipStream_t st) {
  if (nnz > 0) hipLaunchKernelGGL(k_csr_colcount, dim3(unsigned((nnz + 255) / 256)), dim3(256), 0, st, col, nnz, cnt);
}
void launch_csr_tplace(const int64_t* rowptr, const int32_t* col, int n, const int64_t* trowptr, int32_t* cur,
                       int64_t* rec, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_csr_tplace, dim3(unsigned(n)), dim3(64), 0, st, rowptr, col, n, trowptr, cur, rec);
}
void launch_csr_tgather(const int64_t* rec, int64_t nnz, const float* val, int32_t* tcol, float* tval,
                        hipStream_t st) {
  if (nnz > 0)
    hipLaunchKernelGGL(k_csr_tgather, dim3(unsigned((nnz + 255) / 256)), dim3(256), 0, st, rec, nnz, val, tcol, tval);
}

int spinv_cap() { return SPINV_CAP; }
int spinv_wmax() { return SPINV_W; }

void launch_spinv_ball(const SpInvJob& J, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_spinv_ball, dim3(unsigned(grid)), dim3(SPINV_BALL_THREADS), 0, st, J);
}

template <typename T>
void launch_spinv_vals(const SpInvJob& J, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_spinv_vals<T>), dim3(unsigned(grid)), dim3(SPINV_CAP), 0, st, J);
}
template void launch_spinv_vals<float>(const SpInvJob&, int, hipStream_t);
template void launch_spinv_vals<double>(const SpInvJob&, int, hipStream_t);

}  // namespace pmchwt
