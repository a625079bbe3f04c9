// Geometric classification tables, built on the device once per geometry:
//  - the near-field pattern of P: BC pairs (i, j) whose support boxes lie
//    within chi of each other (the cutoff of Section 3.3), as a CSR with
//    ascending columns, found through a uniform grid on the box centres;
//  - the dual-cell pair tables of the near-field BC kernel: every pair of
//    dual cells (v, w) that some kept (i, j) joins, with an N_v x N_w table of
//    CSR positions (-1 where the cutoff dropped the pair);
//  - the singular pairs of A (ordered triangle pairs sharing a vertex, the
//    Sauter-Schwab classes), grouped by test triangle;
//  - the correction tables of the symmetric-tile storage of A;
//  - the number of regular pairs per distance class (work counters).
// Every table is a count pass, a scan and a fill pass; lists are sorted in
// LDS so that the result does not depend on the order of atomic updates.
#include "common.hpp"
#include "kernels.hpp"

namespace pmchwt {

constexpr int CP_CAP = 4096;  // distinct partner cells of one dual cell (LDS hash set)

__global__ void k_cls_fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

// out[i] = float(in[i]) (rounded to nearest)
__global__ void k_d2f(const double* in, float* out, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    out[i] = float(in[i]);
}

void launch_d2f(const double* in, float* out, int64_t n, hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(k_d2f, dim3(unsigned(std::min<int64_t>(4096, (n + 255) / 256))), dim3(256), 0, st, in, out, n);
}

__global__ void k_cls_set_i64(int64_t* p, int64_t v) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *p = v;
}

// Bitonic sort of n keys (a power of two) in LDS by the whole workgroup.
template <typename K>
__device__ void wg_bitonic(K* a, int n) {
  for (int k = 2; k <= n; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int l = i ^ j;
        if (l > i) {
          const K x = a[i], y = a[l];
          if ((x > y) == ((i & k) == 0)) {
            a[i] = y;
            a[l] = x;
          }
        }
      }
      __syncthreads();
    }
}

__device__ __forceinline__ int pow2_at_least(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// Sum over the workgroup (blockDim.x a multiple of 64, at most 1024).
template <typename T>
__device__ T wg_sum(T v) {
  __shared__ T part[16];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) part[w] = v;
  __syncthreads();
  T s = 0;
  for (int q = 0; q < nw; ++q) s += part[q];
  return s;
}

// ---------------------------------------------------------------------------
// Near-field pattern of P
// ---------------------------------------------------------------------------

// Distance of the support boxes of i and j (lo[3], hi[3] each) against chi,
// evaluated as plain IEEE operations (no contraction): per axis the gap
// max(0, lo_j - hi_i, lo_i - hi_j), then sqrt of the sum of squares.
__device__ __forceinline__ bool boxes_within(const double* bi, const double* bj, double chi) {
#pragma clang fp contract(off)
  double g2 = 0.0;
  for (int d = 0; d < 3; ++d) {
    const double g = fmax(0.0, fmax(bj[d] - bi[3 + d], bi[d] - bj[3 + d]));
    g2 = g2 + g * g;
  }
  return sqrt(g2) <= chi;
}

__device__ __forceinline__ void grid_coords(const double* b, const NfGrid& g, int* ijk) {
  for (int d = 0; d < 3; ++d) {
    const double u = floor((0.5 * (b[d] + b[3 + d]) - g.gmin[d]) / g.h);
    ijk[d] = int(fmin(fmax(u, 0.0), double(g.dims[d] - 1)));
  }
}

__global__ void k_nf_bin_count(const double* box, int E, NfGrid g, int32_t* gcell, int32_t* gcnt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  double b[6];
  for (int q = 0; q < 6; ++q) b[q] = box[6 * int64_t(e) + q];
  int ijk[3];
  grid_coords(b, g, ijk);
  const int c = (ijk[0] * g.dims[1] + ijk[1]) * g.dims[2] + ijk[2];
  gcell[e] = c;
  atomicAdd(&gcnt[c], 1);
}

__global__ void k_nf_bin_fill(const int32_t* gcell, int E, const int64_t* gstart, int32_t* gcur, int32_t* gitem) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int c = gcell[e];
  gitem[gstart[c] + atomicAdd(&gcur[c], 1)] = e;
}

// Visits the kept columns of row i among the 27 grid cells around its own;
// `f(j)` is called once per kept j (order unspecified).  Threads of the
// caller split each cell's items by `lane`, stepping by `step`.
template <typename Fn>
__device__ __forceinline__ void nf_row_visit(int i, const NfJob& J, int lane, int step, Fn&& f) {
  double bi[6];
  for (int q = 0; q < 6; ++q) bi[q] = J.box[6 * int64_t(i) + q];
  const int si = J.escat[i];
  const int c = J.gcell[i];
  const int z0 = c % J.g.dims[2], y0 = (c / J.g.dims[2]) % J.g.dims[1], x0 = c / (J.g.dims[2] * J.g.dims[1]);
  for (int x = max(0, x0 - 1); x <= min(J.g.dims[0] - 1, x0 + 1); ++x)
    for (int y = max(0, y0 - 1); y <= min(J.g.dims[1] - 1, y0 + 1); ++y)
      for (int z = max(0, z0 - 1); z <= min(J.g.dims[2] - 1, z0 + 1); ++z) {
        const int cc = (x * J.g.dims[1] + y) * J.g.dims[2] + z;
        for (int64_t p = J.gstart[cc] + lane; p < J.gstart[cc + 1]; p += step) {
          const int j = J.gitem[p];
          if (!J.cross && J.escat[j] != si) continue;
          double bj[6];
          for (int q = 0; q < 6; ++q) bj[q] = J.box[6 * int64_t(j) + q];
          if (boxes_within(bi, bj, J.chi)) f(j);
        }
      }
}

// one wavefront per row: number of kept columns
__global__ __launch_bounds__(256) void k_nf_count(NfJob J, int32_t* cnt, int32_t* maxcnt) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= J.E) return;
  int n = 0;
  nf_row_visit(i, J, lane, 64, [&](int) { ++n; });
  for (int off = 32; off > 0; off >>= 1) n += __shfl_xor(n, off);
  if (lane == 0) {
    cnt[i] = n;
    atomicMax(maxcnt, n);
  }
}

// one workgroup per row: kept columns gathered in LDS (cap entries, a power
// of two at least the longest row), sorted, written at rowptr[i]
__global__ __launch_bounds__(256) void k_nf_fill(NfJob J, const int64_t* rowptr, int cap, int32_t* col) {
  extern __shared__ int32_t s_keys[];
  __shared__ int s_n;
  const int i = blockIdx.x;
  if (threadIdx.x == 0) s_n = 0;
  __syncthreads();
  nf_row_visit(i, J, threadIdx.x, blockDim.x, [&](int j) {
    const int q = atomicAdd(&s_n, 1);
    if (q < cap) s_keys[q] = j;
  });
  __syncthreads();
  const int n = min(s_n, cap);
  const int np = pow2_at_least(n);
  for (int t = n + threadIdx.x; t < np; t += blockDim.x) s_keys[t] = INT32_MAX;
  __syncthreads();
  wg_bitonic(s_keys, np);
  const int64_t base = rowptr[i];
  for (int t = threadIdx.x; t < n; t += blockDim.x) col[base + t] = s_keys[t];
}

// chi < 0: every column of the own scatterer (all columns when cross)
__global__ void k_nf_dense_count(int E, const int32_t* escat, const int32_t* sc_first, const int32_t* sc_n, int cross,
                                 int32_t* cnt, int32_t* maxcnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= E) return;
  const int n = cross ? E : sc_n[escat[i]];
  cnt[i] = n;
  atomicMax(maxcnt, n);
}

__global__ void k_nf_dense_fill(int E, const int32_t* escat, const int32_t* sc_first, int cross, const int64_t* rowptr,
                                int32_t* col) {
  const int i = blockIdx.x;
  const int first = cross ? 0 : sc_first[escat[i]];
  const int64_t b = rowptr[i], n = rowptr[i + 1] - b;
  for (int64_t t = threadIdx.x; t < n; t += blockDim.x) col[b + t] = first + int32_t(t);
}

// ---------------------------------------------------------------------------
// Dual-cell pair tables of the near-field kernel
// ---------------------------------------------------------------------------

// one workgroup per dual cell v.  Partner cells w: the two end cells of every
// column j of the rows i incident to v, deduplicated in an LDS hash set and
// sorted.  FILL = false: counts (pairs, slots); FILL = true: the tables.
template <bool FILL>
__global__ __launch_bounds__(256) void k_cell_pairs(CellPairJob J) {
  __shared__ int32_t s_hash[CP_CAP];  // hash set; after the sort: prefix sums of N_w
  __shared__ int32_t s_list[CP_CAP];
  __shared__ int s_n, s_over;
  __shared__ int32_t s_part[256];
  const int cv = blockIdx.x;
  const int tid = threadIdx.x;
  for (int t = tid; t < CP_CAP; t += blockDim.x) s_hash[t] = -1;
  if (tid == 0) {
    s_n = 0;
    s_over = 0;
  }
  __syncthreads();
  const int e0 = J.inc_ptr[cv], Nv = J.inc_ptr[cv + 1] - e0;
  for (int si = 0; si < Nv; ++si) {
    const int i = J.inc_edges[e0 + si];
    for (int64_t p = J.rowptr[i] + tid; p < J.rowptr[i + 1]; p += blockDim.x) {
      const int j = J.col[p];
      for (int b = 0; b < 2; ++b) {
        const int key = J.ecell[2 * int64_t(j) + b];
        uint32_t h = (uint32_t(key) * 2654435761u) >> 20;  // 12 bits: CP_CAP slots
        int probe = 0;
        for (; probe < CP_CAP; ++probe) {
          const int old = atomicCAS(&s_hash[h], -1, key);
          if (old == -1) {
            const int q = atomicAdd(&s_n, 1);
            if (q < CP_CAP) s_list[q] = key;
            if (q >= CP_CAP * 3 / 4) s_over = 1;
            break;
          }
          if (old == key) break;
          h = (h + 1) & (CP_CAP - 1);
        }
        if (probe == CP_CAP) s_over = 1;
      }
    }
    __syncthreads();
    if (s_over) break;
  }
  __syncthreads();
  if (s_over) {
    if (!FILL && tid == 0) {
      J.ncw[cv] = 0;
      J.nslot[cv] = 0;
      atomicMax(J.flag, 1);
    }
    return;
  }
  const int n = s_n, np = pow2_at_least(n);
  for (int t = n + tid; t < np; t += blockDim.x) s_list[t] = INT32_MAX;
  __syncthreads();
  wg_bitonic(s_list, np);
  // N_w of every partner, as chunk sums per thread then an exclusive scan
  const int per = (n + int(blockDim.x) - 1) / int(blockDim.x);
  const int k0 = min(n, tid * per), k1 = min(n, k0 + per);
  int loc = 0;
  for (int k = k0; k < k1; ++k) loc += J.inc_ptr[s_list[k] + 1] - J.inc_ptr[s_list[k]];
  s_part[tid] = loc;
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int t = 0; t < int(blockDim.x); ++t) {
      const int v = s_part[t];
      s_part[t] = run;
      run += v;
    }
    s_hash[n] = run;  // total over all partners
  }
  __syncthreads();
  {
    int run = s_part[tid];
    for (int k = k0; k < k1; ++k) {
      s_hash[k] = run;
      run += J.inc_ptr[s_list[k] + 1] - J.inc_ptr[s_list[k]];
    }
  }
  __syncthreads();
  const int S = s_hash[n];
  if (!FILL) {
    if (tid == 0) {
      J.ncw[cv] = n;
      J.nslot[cv] = Nv * S;
    }
    return;
  }
  const int64_t pbase = J.pairoff[cv], sbase = J.slotbase[cv];
  for (int k = tid; k < n; k += blockDim.x) {
    J.cpairs[2 * (pbase + k)] = cv;
    J.cpairs[2 * (pbase + k) + 1] = s_list[k];
    J.slot_off[pbase + k] = sbase + int64_t(Nv) * s_hash[k];
  }
  const int total = Nv * S;
  for (int s = tid; s < total; s += blockDim.x) {
    // partner k: Nv * pre[k] <= s < Nv * pre[k + 1]
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (Nv * s_hash[mid] <= s)
        lo = mid;
      else
        hi = mid - 1;
    }
    const int cw = s_list[lo];
    const int w0 = J.inc_ptr[cw], Nw = J.inc_ptr[cw + 1] - w0;
    const int local = s - Nv * s_hash[lo];
    const int si = local / Nw, sj = local - si * Nw;
    const int i = J.inc_edges[e0 + si], j = J.inc_edges[w0 + sj];
    int64_t a = J.rowptr[i], b = J.rowptr[i + 1];  // first column >= j
    while (a < b) {
      const int64_t m = (a + b) >> 1;
      if (J.col[m] < j)
        a = m + 1;
      else
        b = m;
    }
    const bool kept = a < J.rowptr[i + 1] && J.col[a] == j;
    J.slot_pos[sbase + s] = kept ? a : -1;
    if (kept) {  // which ends of i and j the cells v and w are
      const int ai = J.ecell[2 * int64_t(i)] == cv ? 0 : 1, bj = J.ecell[2 * int64_t(j)] == cw ? 0 : 1;
      J.entry_slots[4 * a + 2 * ai + bj] = sbase + s;
    }
  }
}

// ---------------------------------------------------------------------------
// Singular pairs of A
// ---------------------------------------------------------------------------

constexpr int SING_NB = 64;  // triangles sharing a vertex with one triangle

// one thread per test triangle f: the triangles sharing a vertex with f
// (itself included), ascending.  FILL = false: counts; FILL = true: pairs
// (f, t) at sptr[f] and the Sauter-Schwab point count of each.
template <bool FILL>
__global__ void k_sing_list(SingListJob J) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= J.F) return;
  int nb[SING_NB];
  int n = 0;
  bool over = false;
  int va[3];
  for (int a = 0; a < 3; ++a) {
    va[a] = J.tvid[a * J.F + f];
    for (int p = J.v2t_ptr[va[a]]; p < J.v2t_ptr[va[a] + 1]; ++p) {
      if (n < SING_NB)
        nb[n++] = J.v2t[p];
      else
        over = true;
    }
  }
  for (int k = 1; k < n; ++k) {  // insertion sort
    const int v = nb[k];
    int q = k - 1;
    while (q >= 0 && nb[q] > v) {
      nb[q + 1] = nb[q];
      --q;
    }
    nb[q + 1] = v;
  }
  int m = 0;
  for (int k = 0; k < n; ++k)
    if (k == 0 || nb[k] != nb[k - 1]) nb[m++] = nb[k];
  if (!FILL) {
    J.cnt[f] = m;
    if (over) atomicMax(J.flag, 1);
    return;
  }
  const int64_t base = J.sptr[f];
  unsigned long long pts = 0;
  for (int k = 0; k < m; ++k) {
    const int t = nb[k];
    J.pairs[2 * (base + k)] = f;
    J.pairs[2 * (base + k) + 1] = t;
    int shared = 0;
    for (int b = 0; b < 3; ++b) {
      const int vb = J.tvid[b * J.F + t];
      shared += (vb == va[0]) + (vb == va[1]) + (vb == va[2]);
    }
    pts += (unsigned long long)J.npts[min(shared, 3)];
  }
  atomicAdd(J.point_pairs, pts);
}

// ---------------------------------------------------------------------------
// Correction tables of the symmetric-tile storage
// ---------------------------------------------------------------------------

// Every local block entry e = 9 q + 3 a + b of singular pair q = (f, g) adds
// to (r, c) = (t2e(f, a), t2e(g, b)).  With J.all, every such e is a record
// (r, c) with item e << 1: the entries the singular pairs touch, for their
// fixed-order sum.  Otherwise, when r and c fall in different tile rows it
// is a record of the correction entry below the diagonal tiles: (r, c) with
// item e << 1 if tile(r) > tile(c), else (c, r) with item (e << 1) | 1 (the
// entry is read transposed).  PASS 0 counts records per row, PASS 1 places
// them (row-grouped, unordered within a row; k_sym_sort orders them).
template <int PASS>
__global__ void k_sym_records(SymRecJob J) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= 9 * J.npairs) return;
  const int64_t q = idx / 9;
  const int ab = int(idx - 9 * q), a = ab / 3, b = ab - 3 * (ab / 3);
  const int f = J.pairs[2 * q], g = J.pairs[2 * q + 1];
  const int r = J.t2e[a * J.F + f], c = J.t2e[b * J.F + g];
  const int tr = r / J.tile, tc = c / J.tile;
  if (!J.all && tr == tc) return;
  const bool lower = J.all || tr > tc;
  const int R = lower ? r : c, C = lower ? c : r;
  const int32_t item = (int32_t(idx) << 1) | (lower ? 0 : 1);
  if (PASS == 0) {
    atomicMax(J.maxrec, atomicAdd(&J.cnt[R], 1) + 1);
  } else {
    const int64_t pos = J.recptr[R] + atomicAdd(&J.cur[R], 1);
    J.rec[pos] = (int64_t(C) << 32) | int64_t(uint32_t(item));
  }
}

// one workgroup per row: its records sorted by (column, item) in LDS; the
// number of distinct columns is the row's entry count
__global__ __launch_bounds__(256) void k_sym_sort(SymRecJob J, int cap) {
  extern __shared__ int64_t s_rec[];
  const int R = blockIdx.x;
  const int64_t b = J.recptr[R];
  const int n = int(J.recptr[R + 1] - b);
  if (n == 0) {
    if (threadIdx.x == 0) J.cnt[R] = 0;
    return;
  }
  const int np = pow2_at_least(n);
  for (int t = threadIdx.x; t < np; t += blockDim.x) s_rec[t] = t < n ? J.rec[b + t] : INT64_MAX;
  __syncthreads();
  wg_bitonic(s_rec, np);
  int first = 0;
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    J.rec[b + t] = s_rec[t];
    first += (t == 0 || (s_rec[t] >> 32) != (s_rec[t - 1] >> 32)) ? 1 : 0;
  }
  const int tot = wg_sum(first);
  if (threadIdx.x == 0) J.cnt[R] = tot;
}

// one thread per row: entries (R, C) in column order, the first record of
// each, and the items in record order
__global__ void k_sym_emit(SymRecJob J) {
  const int R = blockIdx.x * blockDim.x + threadIdx.x;
  if (R >= J.n) return;
  int64_t k = J.rowptr[R];
  const int64_t b = J.recptr[R], e = J.recptr[R + 1];
  int prev = -1;
  for (int64_t t = b; t < e; ++t) {
    const int64_t v = J.rec[t];
    const int C = int(v >> 32);
    if (C != prev) {
      J.crow[k] = R;
      J.col[k] = C;
      J.iptr[k] = t;
      ++k;
      prev = C;
    }
    J.item[t] = int32_t(uint32_t(v & 0xffffffffll));
  }
}

// ---------------------------------------------------------------------------
// Regular-pair counts per class (work counters)
// ---------------------------------------------------------------------------

// Unordered disjoint pairs (a < b) of the whole union, each counted twice
// (both orientations are integrated), with the point pairs of its class
// rule; grid (test blocks, trial slices).
__global__ __launch_bounds__(256) void k_count_regular(int F, const double* tcen, const double* tdiam2,
                                                       const int32_t* tvid, int n_near, int n_medium, int n_far,
                                                       unsigned long long* out) {
  __shared__ double s_c[256][4];
  __shared__ int32_t s_v[256][3];
  const int a = blockIdx.x * 256 + threadIdx.x;
  const bool live = a < F;
  double ca[3] = {0, 0, 0}, da = 0;
  int va[3] = {-1, -1, -1};
  if (live) {
    for (int d = 0; d < 3; ++d) ca[d] = tcen[d * F + a];
    da = tdiam2[a];
    for (int k = 0; k < 3; ++k) va[k] = tvid[k * F + a];
  }
  const int slice = (F + gridDim.y - 1) / gridDim.y;
  const int b0 = blockIdx.y * slice, b1 = min(F, b0 + slice);
  const int np[3] = {n_near * n_near, n_medium * n_medium, n_far * n_far};
  unsigned long long pairs = 0, pts = 0;
  for (int t0 = b0; t0 < b1; t0 += 256) {
    const int nt = min(256, b1 - t0);
    __syncthreads();
    if (threadIdx.x < nt) {
      const int b = t0 + threadIdx.x;
      for (int d = 0; d < 3; ++d) s_c[threadIdx.x][d] = tcen[d * F + b];
      s_c[threadIdx.x][3] = tdiam2[b];
      for (int k = 0; k < 3; ++k) s_v[threadIdx.x][k] = tvid[k * F + b];
    }
    __syncthreads();
    if (!live) continue;
    for (int t = 0; t < nt; ++t) {
      if (t0 + t <= a) continue;
      bool sh = false;
      for (int k = 0; k < 3; ++k) sh |= (s_v[t][k] == va[0]) | (s_v[t][k] == va[1]) | (s_v[t][k] == va[2]);
      if (sh) continue;
      const int cls = classify_pair(ca[0], ca[1], ca[2], s_c[t][0], s_c[t][1], s_c[t][2], da, s_c[t][3]);
      pairs += 2;
      pts += 2ull * (unsigned long long)np[cls];
    }
  }
  const unsigned long long sp = wg_sum(pairs), spt = wg_sum(pts);
  if (threadIdx.x == 0) {
    atomicAdd(&out[0], sp);
    atomicAdd(&out[1], spt);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static unsigned blocks_for(int64_t n, int per) { return unsigned((n + per - 1) / per); }

void launch_cls_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_cls_fill_i32, dim3(unsigned(std::min<int64_t>(1024, (n + 255) / 256))), dim3(256), 0, st, p, n,
                     v);
}

void launch_cls_set_i64(int64_t* p, int64_t v, hipStream_t st) {
  hipLaunchKernelGGL(k_cls_set_i64, dim3(1), dim3(64), 0, st, p, v);
}

void launch_scan_i32(const int32_t* cnt, int n, int64_t* rowptr, hipStream_t st) {
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, st, cnt, n, rowptr);
}

void launch_nf_bin(const double* box, int E, const NfGrid& g, int32_t* gcell, int32_t* gcnt, hipStream_t st) {
  if (E > 0) hipLaunchKernelGGL(k_nf_bin_count, dim3(blocks_for(E, 256)), dim3(256), 0, st, box, E, g, gcell, gcnt);
}

void launch_nf_bin_fill(const int32_t* gcell, int E, const int64_t* gstart, int32_t* gcur, int32_t* gitem,
                        hipStream_t st) {
  if (E > 0)
    hipLaunchKernelGGL(k_nf_bin_fill, dim3(blocks_for(E, 256)), dim3(256), 0, st, gcell, E, gstart, gcur, gitem);
}

void launch_nf_count(const NfJob& J, int32_t* cnt, int32_t* maxcnt, hipStream_t st) {
  if (J.E > 0) hipLaunchKernelGGL(k_nf_count, dim3(blocks_for(J.E, 4)), dim3(256), 0, st, J, cnt, maxcnt);
}

void launch_nf_fill(const NfJob& J, const int64_t* rowptr, int cap, int32_t* col, hipStream_t st) {
  if (J.E > 0)
    hipLaunchKernelGGL(k_nf_fill, dim3(unsigned(J.E)), dim3(256), size_t(cap) * sizeof(int32_t), st, J, rowptr, cap,
                       col);
}

void launch_nf_dense(int E, const int32_t* escat, const int32_t* sc_first, const int32_t* sc_n, int cross,
                     int32_t* cnt, int32_t* maxcnt, hipStream_t st) {
  if (E > 0)
    hipLaunchKernelGGL(k_nf_dense_count, dim3(blocks_for(E, 256)), dim3(256), 0, st, E, escat, sc_first, sc_n, cross,
                       cnt, maxcnt);
}

void launch_nf_dense_fill(int E, const int32_t* escat, const int32_t* sc_first, int cross, const int64_t* rowptr,
                          int32_t* col, hipStream_t st) {
  if (E > 0)
    hipLaunchKernelGGL(k_nf_dense_fill, dim3(unsigned(E)), dim3(256), 0, st, E, escat, sc_first, cross, rowptr, col);
}

void launch_cell_pairs(const CellPairJob& J, int ncell, bool fill, hipStream_t st) {
  if (ncell <= 0) return;
  if (fill)
    hipLaunchKernelGGL(k_cell_pairs<true>, dim3(unsigned(ncell)), dim3(256), 0, st, J);
  else
    hipLaunchKernelGGL(k_cell_pairs<false>, dim3(unsigned(ncell)), dim3(256), 0, st, J);
}

void launch_sing_list(const SingListJob& J, bool fill, hipStream_t st) {
  if (J.F <= 0) return;
  if (fill)
    hipLaunchKernelGGL(k_sing_list<true>, dim3(blocks_for(J.F, 128)), dim3(128), 0, st, J);
  else
    hipLaunchKernelGGL(k_sing_list<false>, dim3(blocks_for(J.F, 128)), dim3(128), 0, st, J);
}

void launch_sym_records(const SymRecJob& J, int pass, hipStream_t st) {
  if (J.npairs <= 0) return;
  const unsigned nb = blocks_for(9 * J.npairs, 256);
  if (pass == 0)
    hipLaunchKernelGGL(k_sym_records<0>, dim3(nb), dim3(256), 0, st, J);
  else
    hipLaunchKernelGGL(k_sym_records<1>, dim3(nb), dim3(256), 0, st, J);
}

void launch_sym_sort(const SymRecJob& J, int cap, hipStream_t st) {
  if (J.n > 0) hipLaunchKernelGGL(k_sym_sort, dim3(unsigned(J.n)), dim3(256), size_t(cap) * sizeof(int64_t), st, J, cap);
}

void launch_sym_emit(const SymRecJob& J, hipStream_t st) {
  if (J.n > 0) hipLaunchKernelGGL(k_sym_emit, dim3(blocks_for(J.n, 256)), dim3(256), 0, st, J);
}

void launch_count_regular(int F, const double* tcen, const double* tdiam2, const int32_t* tvid, int n_near,
                          int n_medium, int n_far, unsigned long long* out, hipStream_t st) {
  if (F <= 0) return;
  const unsigned gx = blocks_for(F, 256);
  const unsigned gy = unsigned(std::max<int64_t>(1, std::min<int64_t>(64, (F + 1023) / 1024)));
  hipLaunchKernelGGL(k_count_regular, dim3(gx, gy), dim3(256), 0, st, F, tcen, tdiam2, tvid, n_near, n_medium, n_far,
                     out);
}

int cell_pair_capacity() { return CP_CAP * 3 / 4; }
int nf_row_capacity() { return 8192; }
int sing_neighbour_capacity() { return SING_NB; }

}  // namespace pmchwt
