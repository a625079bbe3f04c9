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
// One workgroup per row: a breadth-first search over M's rows builds the ball
// in an LDS hash table, the ball's columns are sorted (the output is a CSR row
// in column order), the gather of (X M)_iq over the column q of M is mapped
// once to local positions (written to a per-workgroup slice of global
// memory), and every Chebyshev step is then a fixed-order gather in LDS:
// deterministic.  Pass 1 only counts the ball of every row (for the CSR row
// pointers); pass 2 computes and writes the values.
#include "common.hpp"
#include "kernels.hpp"

namespace pmchwt {

constexpr int SPINV_THREADS = 256;

__device__ __forceinline__ uint32_t spinv_hash(int32_t j, int mask) {
  return (uint32_t(j) * 2654435761u >> 7) & uint32_t(mask);
}

// LDS layout: keys[H] int32 | pos[H] int16 | cols[CAP] int32 | x, d, r [CAP] double
struct SpInvLds {
  int32_t* keys;
  int16_t* pos;
  int32_t* cols;
  double *x, *d, *r;
  __device__ SpInvLds(unsigned char* raw, int H, int CAP) {
    keys = reinterpret_cast<int32_t*>(raw);
    pos = reinterpret_cast<int16_t*>(raw + 4 * size_t(H));
    cols = reinterpret_cast<int32_t*>(raw + 6 * size_t(H));
    double* base = reinterpret_cast<double*>(raw + ((6 * size_t(H) + 4 * size_t(CAP) + 15) & ~size_t(15)));
    x = base;
    d = base + CAP;
    r = base + 2 * CAP;
  }
};

size_t spinv_lds_bytes(int H, int CAP, bool values) {
  const size_t head = (6 * size_t(H) + 4 * size_t(CAP) + 15) & ~size_t(15);
  return values ? head + 24 * size_t(CAP) : head;
}

// ball of row i: keys / cols filled, returns its size, or -1 past CAP
__device__ int spinv_ball(const SpInvJob& J, int i, SpInvLds& L, int* s_cnt, int* s_over) {
  const int H = J.hash, CAP = J.cap;
  for (int s = threadIdx.x; s < H; s += SPINV_THREADS) L.keys[s] = -1;
  if (threadIdx.x == 0) {
    *s_cnt = 0;
    *s_over = 0;
  }
  __syncthreads();
  auto insert = [&](int32_t j) {
    if (*(volatile int*)s_cnt >= CAP) {  // past the capacity: stop growing (the row is refused)
      *s_over = 1;
      return;
    }
    uint32_t slot = spinv_hash(j, H - 1);
    for (int probe = 0; probe < H; ++probe) {
      const int32_t prev = atomicCAS(&L.keys[slot], -1, j);
      if (prev == -1) {
        const int idx = atomicAdd(s_cnt, 1);
        if (idx < CAP)
          L.cols[idx] = j;
        else
          *s_over = 1;
        return;
      }
      if (prev == j) return;
      slot = (slot + 1) & uint32_t(H - 1);
    }
    *s_over = 1;
  };
  if (threadIdx.x == 0) insert(i);
  __syncthreads();
  int lo = 0, hi = 1;
  for (int lv = 0; lv < J.hops; ++lv) {
    for (int p = lo + threadIdx.x; p < hi; p += SPINV_THREADS) {
      const int jp = L.cols[p];
      for (int64_t e = J.rp[jp]; e < J.rp[jp + 1]; ++e) insert(J.ci[e]);
    }
    __syncthreads();
    lo = hi;
    hi = min(*s_cnt, CAP);
    const bool over = *s_over != 0;
    __syncthreads();
    if (over) return -1;
  }
  return hi;
}

__device__ __forceinline__ int spinv_find(const SpInvLds& L, int H, int32_t j) {
  uint32_t slot = spinv_hash(j, H - 1);
  for (int probe = 0; probe < H; ++probe) {
    const int32_t k = L.keys[slot];
    if (k == j) return L.pos[slot];
    if (k == -1) return -1;
    slot = (slot + 1) & uint32_t(H - 1);
  }
  return -1;
}

__global__ __launch_bounds__(SPINV_THREADS) void k_spinv_count(SpInvJob J) {
  extern __shared__ __align__(16) unsigned char spinv_raw[];
  __shared__ int s_cnt, s_over;
  SpInvLds L(spinv_raw, J.hash, J.cap);
  for (int i = blockIdx.x; i < J.n; i += gridDim.x) {
    const int B = spinv_ball(J, i, L, &s_cnt, &s_over);
    if (threadIdx.x == 0) J.count[i] = B;
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(SPINV_THREADS) void k_spinv_rows(SpInvJob J) {
  extern __shared__ __align__(16) unsigned char spinv_raw[];
  __shared__ int s_cnt, s_over;
  __shared__ double s_red[SPINV_THREADS / WAVE];
  SpInvLds L(spinv_raw, J.hash, J.cap);
  const int H = J.hash;
  int16_t* adj = J.adj + int64_t(blockIdx.x) * J.cap * J.wmax;
  T* oval = static_cast<T*>(J.oval);
  for (int i = blockIdx.x; i < J.n; i += gridDim.x) {
    const int B = spinv_ball(J, i, L, &s_cnt, &s_over);
    if (B < 0) {  // refused in pass 1 already; the host does not use this result
      __syncthreads();
      continue;
    }
    // bitonic sort of the ball's columns (padded with INT_MAX to a power of two)
    int P = 1;
    while (P < B) P <<= 1;
    for (int p = B + threadIdx.x; p < P; p += SPINV_THREADS) L.cols[p] = 0x7fffffff;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1)
      for (int jj = k >> 1; jj > 0; jj >>= 1) {
        for (int t = threadIdx.x; t < P; t += SPINV_THREADS) {
          const int u = t ^ jj;
          if (u > t) {
            const int32_t a = L.cols[t], b = L.cols[u];
            const bool up = (t & k) == 0;
            if ((a > b) == up) {
              L.cols[t] = b;
              L.cols[u] = a;
            }
          }
        }
        __syncthreads();
      }
    // hash slot -> sorted position
    for (int q = threadIdx.x; q < B; q += SPINV_THREADS) {
      const int32_t j = L.cols[q];
      uint32_t slot = spinv_hash(j, H - 1);
      for (int probe = 0; probe < H; ++probe) {
        if (L.keys[slot] == j) {
          L.pos[slot] = int16_t(q);
          break;
        }
        slot = (slot + 1) & uint32_t(H - 1);
      }
    }
    __syncthreads();
    // gather map: for column q of the ball, the local position of every row
    // p of column cols[q] of M (-1 outside the ball), in M's column order
    for (int q = threadIdx.x; q < B; q += SPINV_THREADS) {
      const int32_t j = L.cols[q];
      const int64_t c0 = J.cp[j], c1 = J.cp[j + 1];
      for (int64_t t = c0; t < c1; ++t) adj[int64_t(q) * J.wmax + (t - c0)] = int16_t(spinv_find(L, H, J.ri[t]));
    }
    // X_1 = D_0 = I / d
    const double dd = 0.5 * (J.a + J.b), cc = 0.5 * (J.b - J.a), sigma = dd / cc;
    for (int q = threadIdx.x; q < B; q += SPINV_THREADS) {
      const double v = L.cols[q] == i ? 1.0 / dd : 0.0;
      L.x[q] = v;
      L.d[q] = v;
    }
    __syncthreads();
    double rho_prev = 1.0 / sigma;
    double rs = 0.0;
    for (int k = 1; k <= J.steps; ++k) {
      const double rho = 1.0 / (2.0 * sigma - rho_prev);
      const double cD = rho * rho_prev, cR = 2.0 * rho / cc;
      rs = 0.0;
      for (int q = threadIdx.x; q < B; q += SPINV_THREADS) {
        const int32_t j = L.cols[q];
        const int64_t c0 = J.cp[j], c1 = J.cp[j + 1];
        const int16_t* aq = adj + int64_t(q) * J.wmax;
        double s = 0.0;
        for (int64_t t = c0; t < c1; ++t) {
          const int lp = aq[t - c0];
          if (lp >= 0) s += L.x[lp] * J.cv[t];
        }
        const double R = (j == i ? 1.0 : 0.0) - s;
        L.r[q] = R;
        rs += R * R;
      }
      __syncthreads();
      for (int q = threadIdx.x; q < B; q += SPINV_THREADS) {
        const double dn = cD * L.d[q] + cR * L.r[q];
        L.d[q] = dn;
        L.x[q] += dn;
      }
      __syncthreads();
      rho_prev = rho;
    }
    // residual of the last step over the ball, fixed-order sum
    for (int o = 32; o >= 1; o >>= 1) rs += __shfl_xor(rs, o, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0) s_red[threadIdx.x / WAVE] = rs;
    const int64_t base = J.orp[i];
    for (int q = threadIdx.x; q < B; q += SPINV_THREADS) {
      J.ocol[base + q] = L.cols[q];
      oval[base + q] = T(L.x[q]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < SPINV_THREADS / WAVE; ++w) t += s_red[w];
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

void launch_spinv_count(const SpInvJob& J, int grid, hipStream_t st) {
  const size_t lds = spinv_lds_bytes(J.hash, J.cap, false);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_spinv_count), hipFuncAttributeMaxDynamicSharedMemorySize,
                            int(lds));
  hipLaunchKernelGGL(k_spinv_count, dim3(unsigned(grid)), dim3(SPINV_THREADS), lds, st, J);
}

template <typename T>
void launch_spinv_rows(const SpInvJob& J, int grid, hipStream_t st) {
  const size_t lds = spinv_lds_bytes(J.hash, J.cap, true);
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_spinv_rows<T>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  hipLaunchKernelGGL((k_spinv_rows<T>), dim3(unsigned(grid)), dim3(SPINV_THREADS), lds, st, J);
}
template void launch_spinv_rows<float>(const SpInvJob&, int, hipStream_t);
template void launch_spinv_rows<double>(const SpInvJob&, int, hipStream_t);

}  // namespace pmchwt
