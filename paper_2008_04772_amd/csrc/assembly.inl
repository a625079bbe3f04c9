// Galerkin assembly of S and C on RWG x RWG (the operators of A).
//
// Every entry is a sum over triangle pairs of int_T1 int_T2 (Section 3.3).
// Disjoint pairs: tensor symmetric triangle rules chosen by relative distance
// (near / medium / far); pairs that share a vertex, an edge or coincide:
// Sauter-Schwab rules.  Each pair accumulates the kernel moments of
// common.hpp once per wavenumber and contracts them against the three RWG
// functions of each triangle; the 3x3 local blocks are scattered into the
// dense matrices, each entry by one thread (regular pairs: the row
// combine; singular pairs: a scatter over their entry tables).
//
// Layout in HBM: one dense row-major matrix per operator, complex
// interleaved (re, im), element type double (FP64) or float (mixed).  The
// exterior operators S^e, C^e span all scatterers (E_tot x E_tot); the
// interior operators S^i_m, C^i_m are separate E_m x E_m matrices.
#include "common.hpp"
#include "kernels.hpp"

namespace pmchwt {

// Symmetric triangle rules: barycentric points and weights (sum 1) of
// degree 1, 2, 3, 4 (1, 3, 4, 6 points): Dunavant, Int. J. Numer. Meth. Eng.
// 21 (1985).  Stored at offsets 0, 1, 4, 8.
__constant__ double c_rule_l[14][3];
__constant__ double c_rule_w[14];
__constant__ int c_rule_off[5] = {0, 0, 1, 4, 8};
__constant__ int c_rule_n[5] = {0, 1, 3, 4, 6};

hipError_t upload_rules(const double* l, const double* w, hipStream_t s) {
  hipError_t e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_rule_l), l, sizeof(double) * 42, 0, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbolAsync(HIP_SYMBOL(c_rule_w), w, sizeof(double) * 14, 0, hipMemcpyHostToDevice, s);
}

// Relative-distance class of a disjoint pair: 0 near, 1 medium, 2 far.
// Evaluated in FP64 without contraction (the pragma marks these operations
// non-fusable, also once inlined) so that it reproduces a plain IEEE
// evaluation of |c1 - c2|^2 < 4 max(d1^2, d2^2) (resp. 16).
__device__ __forceinline__ int classify_pair(double c1x, double c1y, double c1z, double c2x, double c2y, double c2z,
                                             double d1, double d2) {
#pragma clang fp contract(off)
  double dx = c1x - c2x, dy = c1y - c2y, dz = c1z - c2z;
  double dist2 = dx * dx + dy * dy + dz * dz;
  double m2 = d1 > d2 ? d1 : d2;
  if (dist2 < 4.0 * m2) return 0;
  if (dist2 < 16.0 * m2) return 1;
  return 2;
}

// ---------------------------------------------------------------------------
// Regular (disjoint) pairs, pass 1: workgroup = (test triangle t1, chunk of
// trial edges).  Phase A integrates the chunk's distinct trial triangles
// against t1 (moments in LDS, zero for pairs sharing a vertex: those are the
// singular kernel's); phase B contracts them for every trial edge of the
// chunk and every RWG function of t1, summing the T+ and T- contributions,
// and stores one complex value per (slot, edge, operator) - coalesced along
// the edges, no atomics.
// ---------------------------------------------------------------------------
template <typename R>
struct MomPair {
  Moments<R> e, i;
};

// Threads per workgroup of the regular kernel; a chunk of trial edges holds at
// most this many distinct trial triangles, so phase A takes one pass.
template <typename R>
struct RegularThreads {
  static constexpr int value = sizeof(R) == 4 ? 256 : 128;
};
int regular_chunk_limit(bool fp64) { return fp64 ? RegularThreads<double>::value : RegularThreads<float>::value; }

template <typename R, typename M>
__global__ __launch_bounds__(RegularThreads<R>::value) void k_regular_rows(AsmParams<M> p, HalfJob<M> h,
                                                                            int t1_base) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  MomPair<R>* sm = reinterpret_cast<MomPair<R>*>(smem_raw);
  const int t1 = t1_base + blockIdx.y;
  const int ch = blockIdx.x;
  if (h.skip_lower && h.ch_tmax[ch] < h.t1_tmin[t1]) return;  // lower tiles only: mirrored later
  const int F = p.F;
  const int l0 = h.chunk_ptr[ch], nl = h.chunk_ptr[ch + 1] - l0;
  const int s1 = p.tscat[t1];
  double c1[3];
  for (int d = 0; d < 3; ++d) c1[d] = p.tcen[d * F + t1];
  int va[3];
  R P1[3][3];
  for (int k = 0; k < 3; ++k) {
    va[k] = p.tvid[k * F + t1];
    for (int d = 0; d < 3; ++d) P1[k][d] = R(p.tv[(3 * k + d) * F + t1] - c1[d]);
  }
  const double A1 = p.tarea[t1], d1 = p.tdiam2[t1];
  const double ke_r = p.k_ext;
  const double ki_r = p.k_int[2 * s1], ki_i = p.k_int[2 * s1 + 1];
  const bool decay_i = ki_i != 0.0;

  // ---- phase A: moments of (t1, T) for every listed trial triangle T
  for (int li = threadIdx.x; li < nl; li += blockDim.x) {
    const int t2 = h.chunk_tri[l0 + li];
    bool shared = false;
    bool done_i = false, done_e = false;
    for (int k = 0; k < 3; ++k) {
      const int vb = p.tvid[k * F + t2];
      shared |= (vb == va[0]) | (vb == va[1]) | (vb == va[2]);
    }
    if (!shared) {
      double c2[3];
      for (int d = 0; d < 3; ++d) c2[d] = p.tcen[d * F + t2];
      const int cls = classify_pair(c1[0], c1[1], c1[2], c2[0], c2[1], c2[2], d1, p.tdiam2[t2]);
      const int q = cls == 0 ? p.q_near : (cls == 1 ? p.q_medium : p.q_far);
      const bool inner = p.tscat[t2] == s1;
      R P2[3][3];
      for (int k = 0; k < 3; ++k)
        for (int d = 0; d < 3; ++d) P2[k][d] = R(p.tv[(3 * k + d) * F + t2] - c1[d]);
      const R AA = R(A1 * p.tarea[t2]);
      const int off = c_rule_off[q], n = c_rule_n[q];
      // FP32: trial-side points and weights of the rule (at most 6) in
      // registers, the innermost loop unrolled with a guard so that it reads
      // no memory.  FP64 keeps the rolled loop (the register copy would spill).
      constexpr bool REG = sizeof(R) == 4;
      R yb[REG ? 6 : 1][3], wb[REG ? 6 : 1];
      if constexpr (REG) {
#pragma unroll
        for (int b = 0; b < 6; ++b) {
          if (b < n) {
            const R lb0 = R(c_rule_l[off + b][0]), lb1 = R(c_rule_l[off + b][1]), lb2 = R(c_rule_l[off + b][2]);
#pragma unroll
            for (int d = 0; d < 3; ++d) yb[b][d] = lb0 * P2[0][d] + lb1 * P2[1][d] + lb2 * P2[2][d];
            wb[b] = R(c_rule_w[off + b]);
          } else {
            yb[b][0] = yb[b][1] = yb[b][2] = wb[b] = R(0);
          }
        }
      }
      // one wavenumber at a time keeps 14 complex accumulators live, not 28
      for (int kk = 0; kk < (inner ? 2 : 1); ++kk) {
        Moments<R> mm;
        mm.zero();
        const R kr = R(kk == 0 ? ke_r : ki_r), ki = R(kk == 0 ? 0.0 : ki_i);
        const bool decay = kk == 0 ? false : decay_i;
#pragma unroll 1
        for (int a = 0; a < n; ++a) {
          R x[3];
          const R la0 = R(c_rule_l[off + a][0]), la1 = R(c_rule_l[off + a][1]), la2 = R(c_rule_l[off + a][2]);
#pragma unroll
          for (int d = 0; d < 3; ++d) x[d] = la0 * P1[0][d] + la1 * P1[1][d] + la2 * P1[2][d];
          const R wa = R(c_rule_w[off + a]) * AA;
          if constexpr (REG) {
#pragma unroll
            for (int b = 0; b < 6; ++b) {
              if (b < n) {
                const R w = wa * wb[b];
                const R dx = x[0] - yb[b][0], dy = x[1] - yb[b][1], dz = x[2] - yb[b][2];
                const R r2 = dx * dx + dy * dy + dz * dz;
                mm.add(helmholtz<R>(r2, kr, ki, decay, w), x, yb[b], true);
              }
            }
          } else {
#pragma unroll 1
            for (int b = 0; b < n; ++b) {
              R y[3];
              const R lb0 = R(c_rule_l[off + b][0]), lb1 = R(c_rule_l[off + b][1]), lb2 = R(c_rule_l[off + b][2]);
#pragma unroll
              for (int d = 0; d < 3; ++d) y[d] = lb0 * P2[0][d] + lb1 * P2[1][d] + lb2 * P2[2][d];
              const R w = wa * R(c_rule_w[off + b]);
              const R dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
              const R r2 = dx * dx + dy * dy + dz * dz;
              mm.add(helmholtz<R>(r2, kr, ki, decay, w), x, y, true);
            }
          }
        }
        if (kk == 0) {
          sm[li].e = mm;
          done_e = true;
        } else {
          sm[li].i = mm;
          done_i = true;
        }
      }
    }
    if (!done_e) sm[li].e.zero();
    if (!done_i) sm[li].i.zero();
  }
  __syncthreads();

  // ---- phase B: one trial edge per thread
  const int j0 = h.chunk_e[ch];
  const int nj = h.chunk_e[ch + 1] - j0;
  R al1[3], w1[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    al1[a] = R(p.tsgn[a * F + t1] / (2.0 * A1));
#pragma unroll
    for (int d = 0; d < 3; ++d) w1[a][d] = al1[a] * P1[a][d];
  }
  const R kre = R(ke_r), kri = R(ki_r), kii = R(ki_i);
  const int64_t slot0 = 3 * int64_t(t1 - h.slab_t0);
  for (int jj = threadIdx.x; jj < nj; jj += blockDim.x) {
    const int j = j0 + jj;
    const int16_t* em = h.edge_map + 4 * int64_t(j);
    const bool inner = h.edge_scat[j] == s1;
    cplx<R> Se[3] = {{0, 0}, {0, 0}, {0, 0}}, Ce[3] = {{0, 0}, {0, 0}, {0, 0}};
    cplx<R> Si[3] = {{0, 0}, {0, 0}, {0, 0}}, Ci[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int side = 0; side < 2; ++side) {
      const int pos = em[2 * side], b = em[2 * side + 1];
      const int t2 = h.chunk_tri[l0 + pos];
      const double A2 = p.tarea[t2];
      const R al2 = R(p.tsgn[b * F + t2] / (2.0 * A2));
      R w2[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) w2[d] = al2 * R(p.tv[(3 * b + d) * F + t2] - c1[d]);
      const MomPair<R>& m = sm[pos];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        cplx<R> S, C;
        contract_r<R>(m.e, al1[a], w1[a], al2, w2, kre, R(0), S, C);
        Se[a].re += S.re;
        Se[a].im += S.im;
        Ce[a].re += C.re;
        Ce[a].im += C.im;
        if (inner) {
          contract_r<R>(m.i, al1[a], w1[a], al2, w2, kri, kii, S, C);
          Si[a].re += S.re;
          Si[a].im += S.im;
          Ci[a].re += C.re;
          Ci[a].im += C.im;
        }
      }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int64_t o = 2 * ((slot0 + a) * h.E_tot + j);
      h.He_S[o] = M(Se[a].re);
      h.He_S[o + 1] = M(Se[a].im);
      h.He_C[o] = M(Ce[a].re);
      h.He_C[o + 1] = M(Ce[a].im);
      if (inner) {
        const int64_t oi = 2 * ((slot0 + a) * h.ld_i + (j - h.edge_off_i));
        h.Hi_S[oi] = M(Si[a].re);
        h.Hi_S[oi + 1] = M(Si[a].im);
        h.Hi_C[oi] = M(Ci[a].re);
        h.Hi_C[oi + 1] = M(Ci[a].im);
      }
    }
  }
}

// Pass 2: A[rows[r]] += H[sp[r]] + H[sm[r]] over complex columns, or with OW
// A[rows[r]] = H[sp[r]] + H[sm[r]] and zero padding columns up to lda (rows
// that no other slab touches: no clearing pass before, same sums).  One
// workgroup per row, striding over its columns in units of U values: U = 1,
// or 16-byte vectors when both rows start on 16-byte boundaries and the
// column counts are whole vectors.
template <typename M, bool OW, int U>
__global__ __launch_bounds__(256) void k_rows_combine(M* A, int64_t lda, const M* __restrict__ H, int64_t ldh,
                                                      const int32_t* rows, const int32_t* sp, const int32_t* sm,
                                                      int ncols, const int32_t* cstart) {
  typedef M VU __attribute__((ext_vector_type(U)));
  const int r = blockIdx.x;
  const int i = rows[r], a = sp[r], b = sm[r];
  VU* Ar = reinterpret_cast<VU*>(A + 2 * int64_t(i) * lda);
  const VU* Ha = reinterpret_cast<const VU*>(H + 2 * int64_t(a >= 0 ? a : 0) * ldh);
  const VU* Hb = reinterpret_cast<const VU*>(H + 2 * int64_t(b >= 0 ? b : 0) * ldh);
  const int64_t nc = 2 * int64_t(ncols) / U, end = OW ? 2 * lda / U : nc;
  const int64_t q0 = cstart ? 2 * int64_t(cstart[r]) / U : 0;
#pragma unroll 4
  for (int64_t q = q0 + threadIdx.x; q < end; q += 256) {
    VU v = OW ? VU(M(0)) : Ar[q];
    if (!OW || q < nc) {
      if (a >= 0) v += Ha[q];
      if (b >= 0) v += Hb[q];
    }
    Ar[q] = v;
  }
}

// ---------------------------------------------------------------------------
// Singular pairs (shared vertex, shared edge, identical): one wavefront per
// ordered pair, lanes stride over the Sauter-Schwab points, FP64 always.
// Reference element That = {0 <= x2 <= x1 <= 1}, x = P0 + x1 (P1-P0) + x2 (P2-P1)
// with the shared vertices first (in the order of the test triangle), then
// the remaining vertex of each triangle; weights include |J| = 2A per side.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

template <typename M>
__global__ __launch_bounds__(256) void k_singular(AsmParams<M> p, SingParams s) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t pair = int64_t(blockIdx.x) * (blockDim.x / WAVE) + (threadIdx.x / WAVE);
  if (pair >= s.npairs) return;
  const int F = p.F;
  const int t1 = s.pairs[2 * pair], t2 = s.pairs[2 * pair + 1];
  int va[3], vb[3];
  for (int k = 0; k < 3; ++k) {
    va[k] = p.tvid[k * F + t1];
    vb[k] = p.tvid[k * F + t2];
  }
  // reorder: common vertices first, in test-triangle order
  int oa, ob;
  const int nc = shared_order(va, vb, oa, ob);
  double c1[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) c1[d] = p.tcen[d * F + t1];
  double P1[3][3], P2[3][3], Q1[3][3], Q2[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      P1[k][d] = p.tv[(3 * k + d) * F + t1] - c1[d];
      P2[k][d] = p.tv[(3 * k + d) * F + t2] - c1[d];
    }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int ia = (oa >> (2 * k)) & 3, ib = (ob >> (2 * k)) & 3;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double u1[3] = {P1[0][d], P1[1][d], P1[2][d]}, u2[3] = {P2[0][d], P2[1][d], P2[2][d]};
      Q1[k][d] = pick3(u1, ia);
      Q2[k][d] = pick3(u2, ib);
    }
  }
  const double A1 = p.tarea[t1], A2 = p.tarea[t2];
  const int sc = p.tscat[t1];
  const double ke_r = p.k_ext;
  const double ki_r = p.k_int[2 * sc], ki_i = p.k_int[2 * sc + 1];
  const bool decay_i = ki_i != 0.0;
  // nc = 1 vertex, 2 edge, 3 identical
  const double* tab = nc == 1 ? s.tab[1] : (nc == 2 ? s.tab[2] : s.tab[3]);
  const int npts = nc == 1 ? s.npts[1] : (nc == 2 ? s.npts[2] : s.npts[3]);
  const double AA = 4.0 * A1 * A2;

  Moments<double> me, mi;
  me.zero();
  mi.zero();
  for (int k = lane; k < npts; k += WAVE) {
    const double x1 = tab[5 * k], x2 = tab[5 * k + 1], y1 = tab[5 * k + 2], y2 = tab[5 * k + 3];
    const double w = tab[5 * k + 4] * AA;
    double x[3], y[3];
    for (int d = 0; d < 3; ++d) {
      x[d] = Q1[0][d] + x1 * (Q1[1][d] - Q1[0][d]) + x2 * (Q1[2][d] - Q1[1][d]);
      y[d] = Q2[0][d] + y1 * (Q2[1][d] - Q2[0][d]) + y2 * (Q2[2][d] - Q2[1][d]);
    }
    const double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
    const double r2 = dx * dx + dy * dy + dz * dz;
    KernelVal<double> kv = helmholtz<double>(r2, ke_r, 0.0, false, w);
    me.add(kv, x, y, true);
    KernelVal<double> kw = helmholtz<double>(r2, ki_r, ki_i, decay_i, w);
    mi.add(kw, x, y, true);
  }
  // wavefront reduction of both moment sets
  double* fe = reinterpret_cast<double*>(&me);
  double* fi = reinterpret_cast<double*>(&mi);
  constexpr int NM = sizeof(Moments<double>) / sizeof(double);
#pragma unroll
  for (int i = 0; i < NM; ++i) {
    fe[i] = wave_sum(fe[i]);
    fi[i] = wave_sum(fi[i]);
  }
  if (lane < 9) {
    const int a = lane / 3, b = lane % 3;
    const double sa = p.tsgn[a * F + t1], sb = p.tsgn[b * F + t2];
    const double al1 = sa / (2.0 * A1), al2 = sb / (2.0 * A2);
    double w1[3], w2[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double u1[3] = {P1[0][d], P1[1][d], P1[2][d]}, u2[3] = {P2[0][d], P2[1][d], P2[2][d]};
      w1[d] = al1 * pick3(u1, a);
      w2[d] = al2 * pick3(u2, b);
    }
    cplx<double> Se, Ce, Si, Ci;
    contract<double, double>(me, al1, w1, al2, w2, ke_r, 0.0, true, Se, Ce);
    contract<double, double>(mi, al1, w1, al2, w2, ki_r, ki_i, true, Si, Ci);
    double* q = s.blk + 8 * (9 * pair + lane);
    q[0] = Se.re;
    q[1] = Se.im;
    q[2] = Ce.re;
    q[3] = Ce.im;
    q[4] = Si.re;
    q[5] = Si.im;
    q[6] = Ci.re;
    q[7] = Ci.im;
  }
}

// One thread per matrix entry (r, c) that singular pairs touch: the sum of
// its local-block entries in the order of the entry tables (pair, then 3a+b),
// added to S^e, C^e (union indices) and S^i, C^i of the scatterer (local
// indices).  Each entry has one writer, so the result does not depend on the
// order in which the pairs were integrated.
template <typename M>
__global__ void k_sing_scatter(AsmParams<M> p, SingParams s) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= s.e_nnz) return;
  const int r = s.e_row[k], c = s.e_col[k];
  const int64_t b = s.e_iptr[k], e = s.e_iptr[k + 1];
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t t = b; t < e; ++t) {
    const double* q = s.blk + 8 * int64_t(uint32_t(s.e_item[t]) >> 1);
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] += q[u];
  }
  const int pr = int((uint32_t(s.e_item[b]) >> 1) / 9);
  const int sc = p.tscat[s.pairs[2 * pr]];
  const int o = p.edge_off[sc];
  M* const mats[4] = {p.Se + 2 * (int64_t(r) * p.ld_ext + c), p.Ce + 2 * (int64_t(r) * p.ld_ext + c),
                      p.Si[sc] + 2 * (int64_t(r - o) * p.ld_int[sc] + (c - o)),
                      p.Ci[sc] + 2 * (int64_t(r - o) * p.ld_int[sc] + (c - o))};
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    mats[m][0] = M(double(mats[m][0]) + v[2 * m]);
    mats[m][1] = M(double(mats[m][1]) + v[2 * m + 1]);
  }
}

template <typename R, typename M>
void launch_regular_rows(const AsmParams<M>& p, const HalfJob<M>& h, int t1_begin, int t1_end, int nchunks,
                         int max_list, hipStream_t st) {
  const size_t lds = size_t(max_list) * sizeof(MomPair<R>);
  for (int t0 = t1_begin; t0 < t1_end; t0 += 65535) {
    const int rows = std::min(65535, t1_end - t0);
    hipLaunchKernelGGL((k_regular_rows<R, M>), dim3(nchunks, rows), dim3(RegularThreads<R>::value), lds, st, p, h,
                       t0);
  }
}

template <typename M>
void launch_rows_combine(M* A, int64_t lda, const M* H, int64_t ldh, const int32_t* rows, const int32_t* sp,
                         const int32_t* sm, int nrows, int ncols, hipStream_t st, bool overwrite,
                         const int32_t* cstart) {
  if (nrows <= 0) return;
  constexpr int U = 16 / sizeof(M);
  // 16-byte units: row starts (2 ldh, 2 lda values apart) and the column
  // counts must be whole units
  const bool vec = (2 * ldh) % U == 0 && (2 * lda) % U == 0 && (2 * int64_t(ncols)) % U == 0;
  const dim3 grid{static_cast<unsigned>(nrows)}, block{256};
  if (vec && overwrite)
    hipLaunchKernelGGL((k_rows_combine<M, true, U>), grid, block, 0, st, A, lda, H, ldh, rows, sp, sm, ncols, cstart);
  else if (vec)
    hipLaunchKernelGGL((k_rows_combine<M, false, U>), grid, block, 0, st, A, lda, H, ldh, rows, sp, sm, ncols,
                       cstart);
  else if (overwrite)
    hipLaunchKernelGGL((k_rows_combine<M, true, 1>), grid, block, 0, st, A, lda, H, ldh, rows, sp, sm, ncols, cstart);
  else
    hipLaunchKernelGGL((k_rows_combine<M, false, 1>), grid, block, 0, st, A, lda, H, ldh, rows, sp, sm, ncols,
                       cstart);
}

template <typename M>
void launch_singular(const AsmParams<M>& p, const SingParams& s, hipStream_t st) {
  if (s.npairs == 0) return;
  const int per_block = 256 / WAVE;
  const int64_t blocks = (s.npairs + per_block - 1) / per_block;
  hipLaunchKernelGGL((k_singular<M>), dim3(unsigned(blocks)), dim3(256), 0, st, p, s);
  if (s.e_nnz > 0)
    hipLaunchKernelGGL((k_sing_scatter<M>), dim3(unsigned((s.e_nnz + 255) / 256)), dim3(256), 0, st, p, s);
}

template void launch_regular_rows<double, double>(const AsmParams<double>&, const HalfJob<double>&, int, int, int,
                                                  int, hipStream_t);
template void launch_regular_rows<float, float>(const AsmParams<float>&, const HalfJob<float>&, int, int, int, int,
                                                hipStream_t);
template void launch_rows_combine<double>(double*, int64_t, const double*, int64_t, const int32_t*, const int32_t*,
                                          const int32_t*, int, int, hipStream_t, bool, const int32_t*);
template void launch_rows_combine<float>(float*, int64_t, const float*, int64_t, const int32_t*, const int32_t*,
                                         const int32_t*, int, int, hipStream_t, bool, const int32_t*);
template void launch_singular<double>(const AsmParams<double>&, const SingParams&, hipStream_t);
template void launch_singular<float>(const AsmParams<float>&, const SingParams&, hipStream_t);

}  // namespace pmchwt
