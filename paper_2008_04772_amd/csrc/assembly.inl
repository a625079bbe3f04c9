// Galerkin assembly of S and C on RWG x RWG (the operators of A).
//
// Every entry is a sum over triangle pairs of int_T1 int_T2 (Section 3.3).
// Disjoint pairs: tensor symmetric triangle rules chosen by relative distance
// (near / medium / far); pairs that share a vertex, an edge or coincide:
// Sauter-Schwab rules.  Each pair accumulates the kernel moments of
// common.hpp once per wavenumber and contracts them against the three RWG
// functions of each triangle; the 3x3 local blocks are scattered into the
// dense matrices with hardware atomics.
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
// Evaluated in FP64 without contraction so that it reproduces a plain
// IEEE evaluation of |c1 - c2|^2 < 4 max(d1^2, d2^2) (resp. 16).
__device__ __noinline__ int classify_pair(const double* c1, const double* c2, double d1, double d2) {
#pragma clang fp contract(off)
  double dx = c1[0] - c2[0], dy = c1[1] - c2[1], dz = c1[2] - c2[2];
  double dist2 = dx * dx + dy * dy + dz * dz;
  double m2 = d1 > d2 ? d1 : d2;
  if (dist2 < 4.0 * m2) return 0;
  if (dist2 < 16.0 * m2) return 1;
  return 2;
}

template <typename M>
__device__ __forceinline__ void add_entry(M* mat, int64_t ld, int i, int j, const cplx<double>& v) {
  M* p = mat + 2 * (int64_t(i) * ld + j);
  atomic_add(p, M(v.re));
  atomic_add(p + 1, M(v.im));
}

// ---------------------------------------------------------------------------
// Regular (disjoint) pairs: one thread per unordered pair t1 < t2.  The
// tensor rule is symmetric in the two triangles, so the (t2, t1) block is the
// transpose of the (t1, t2) block and is written from the same moments.
// ---------------------------------------------------------------------------
template <typename R, typename M>
__global__ __launch_bounds__(256) void k_regular(AsmParams<M> p, int t1_base) {
  const int t1 = t1_base + blockIdx.y;
  const int t2 = blockIdx.x * blockDim.x + threadIdx.x;
  if (t2 >= p.F || t2 <= t1) return;
  const int F = p.F;
  int va[3], vb[3];
  for (int k = 0; k < 3; ++k) {
    va[k] = p.tvid[k * F + t1];
    vb[k] = p.tvid[k * F + t2];
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      if (va[i] == vb[j]) return;  // singular pair: handled by k_singular

  double c1[3], c2[3];
  for (int d = 0; d < 3; ++d) {
    c1[d] = p.tcen[d * F + t1];
    c2[d] = p.tcen[d * F + t2];
  }
  const int cls = classify_pair(c1, c2, p.tdiam2[t1], p.tdiam2[t2]);
  const int q = cls == 0 ? p.q_near : (cls == 1 ? p.q_medium : p.q_far);
  const int s1 = p.tscat[t1], s2 = p.tscat[t2];
  const bool inner = (s1 == s2);

  // vertex coordinates relative to the test centroid (local origin)
  R P1[3][3], P2[3][3];
  for (int k = 0; k < 3; ++k)
    for (int d = 0; d < 3; ++d) {
      P1[k][d] = R(p.tv[(3 * k + d) * F + t1] - c1[d]);
      P2[k][d] = R(p.tv[(3 * k + d) * F + t2] - c1[d]);
    }
  const double A1 = p.tarea[t1], A2 = p.tarea[t2];
  const double ke_r = p.k_ext;
  const double ki_r = inner ? p.k_int[2 * s1] : 0.0, ki_i = inner ? p.k_int[2 * s1 + 1] : 0.0;
  const bool decay_i = ki_i != 0.0;

  Moments<R> me, mi;
  me.zero();
  mi.zero();
  const int off = c_rule_off[q], n = c_rule_n[q];
  const R AA = R(A1 * A2);
  for (int a = 0; a < n; ++a) {
    R x[3];
    const R la0 = R(c_rule_l[off + a][0]), la1 = R(c_rule_l[off + a][1]), la2 = R(c_rule_l[off + a][2]);
    for (int d = 0; d < 3; ++d) x[d] = la0 * P1[0][d] + la1 * P1[1][d] + la2 * P1[2][d];
    const R wa = R(c_rule_w[off + a]) * AA;
    for (int b = 0; b < n; ++b) {
      R y[3];
      const R lb0 = R(c_rule_l[off + b][0]), lb1 = R(c_rule_l[off + b][1]), lb2 = R(c_rule_l[off + b][2]);
      for (int d = 0; d < 3; ++d) y[d] = lb0 * P2[0][d] + lb1 * P2[1][d] + lb2 * P2[2][d];
      const R w = wa * R(c_rule_w[off + b]);
      const R dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
      const R r2 = dx * dx + dy * dy + dz * dz;
      KernelVal<R> kv = helmholtz<R>(r2, R(ke_r), R(0), false, w);
      me.add(kv, x, y, true);
      if (inner) {
        KernelVal<R> kw = helmholtz<R>(r2, R(ki_r), R(ki_i), decay_i, w);
        mi.add(kw, x, y, true);
      }
    }
  }
  // epilogue: RT0 coefficients of the local RWG functions, u = alpha x - w
  double al1[3], w1[3][3], al2[3], w2[3][3];
  for (int a = 0; a < 3; ++a) {
    const double sa = p.tsgn[a * F + t1], sb = p.tsgn[a * F + t2];
    al1[a] = sa / (2.0 * A1);
    al2[a] = sb / (2.0 * A2);
    for (int d = 0; d < 3; ++d) {
      w1[a][d] = al1[a] * double(P1[a][d]);
      w2[a][d] = al2[a] * double(P2[a][d]);
    }
  }
  int e1[3], e2[3];
  for (int a = 0; a < 3; ++a) {
    e1[a] = p.t2e[a * F + t1];
    e2[a] = p.t2e[a * F + t2];
  }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      cplx<double> S, C;
      contract<R, double>(me, al1[a], w1[a], al2[b], w2[b], ke_r, 0.0, true, S, C);
      add_entry(p.Se, p.ld_ext, e1[a], e2[b], S);
      add_entry(p.Se, p.ld_ext, e2[b], e1[a], S);
      add_entry(p.Ce, p.ld_ext, e1[a], e2[b], C);
      add_entry(p.Ce, p.ld_ext, e2[b], e1[a], C);
      if (inner) {
        contract<R, double>(mi, al1[a], w1[a], al2[b], w2[b], ki_r, ki_i, true, S, C);
        const int o = p.edge_off[s1];
        const int64_t ld = p.ld_int[s1];
        M* Si = p.Si[s1];
        M* Ci = p.Ci[s1];
        add_entry(Si, ld, e1[a] - o, e2[b] - o, S);
        add_entry(Si, ld, e2[b] - o, e1[a] - o, S);
        add_entry(Ci, ld, e1[a] - o, e2[b] - o, C);
        add_entry(Ci, ld, e2[b] - o, e1[a] - o, C);
      }
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
  int oa[3], ob[3], nc = 0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      if (va[i] == vb[j]) {
        oa[nc] = i;
        ob[nc] = j;
        ++nc;
      }
  {
    int ka = nc, kb = nc;
    for (int i = 0; i < 3; ++i) {
      bool c = false;
      for (int j = 0; j < nc; ++j) c |= (oa[j] == i);
      if (!c) oa[ka++] = i;
    }
    for (int i = 0; i < 3; ++i) {
      bool c = false;
      for (int j = 0; j < nc; ++j) c |= (ob[j] == i);
      if (!c) ob[kb++] = i;
    }
  }
  double c1[3];
  for (int d = 0; d < 3; ++d) c1[d] = p.tcen[d * F + t1];
  double P1[3][3], P2[3][3], Q1[3][3], Q2[3][3];
  for (int k = 0; k < 3; ++k)
    for (int d = 0; d < 3; ++d) {
      P1[k][d] = p.tv[(3 * k + d) * F + t1] - c1[d];
      P2[k][d] = p.tv[(3 * k + d) * F + t2] - c1[d];
    }
  for (int k = 0; k < 3; ++k)
    for (int d = 0; d < 3; ++d) {
      Q1[k][d] = P1[oa[k]][d];
      Q2[k][d] = P2[ob[k]][d];
    }
  const double A1 = p.tarea[t1], A2 = p.tarea[t2];
  const int sc = p.tscat[t1];
  const double ke_r = p.k_ext;
  const double ki_r = p.k_int[2 * sc], ki_i = p.k_int[2 * sc + 1];
  const bool decay_i = ki_i != 0.0;
  const int kind = nc;  // 1 vertex, 2 edge, 3 identical
  const double* tab = s.tab[kind];
  const int npts = s.npts[kind];
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
  for (int i = 0; i < NM; ++i) {
    fe[i] = wave_sum(fe[i]);
    fi[i] = wave_sum(fi[i]);
  }
  if (lane < 9) {
    const int a = lane / 3, b = lane % 3;
    const double sa = p.tsgn[a * F + t1], sb = p.tsgn[b * F + t2];
    const double al1 = sa / (2.0 * A1), al2 = sb / (2.0 * A2);
    double w1[3], w2[3];
    for (int d = 0; d < 3; ++d) {
      w1[d] = al1 * P1[a][d];
      w2[d] = al2 * P2[b][d];
    }
    const int i = p.t2e[a * F + t1], j = p.t2e[b * F + t2];
    cplx<double> S, C;
    contract<double, double>(me, al1, w1, al2, w2, ke_r, 0.0, true, S, C);
    add_entry(p.Se, p.ld_ext, i, j, S);
    add_entry(p.Ce, p.ld_ext, i, j, C);
    contract<double, double>(mi, al1, w1, al2, w2, ki_r, ki_i, true, S, C);
    const int o = p.edge_off[sc];
    add_entry(p.Si[sc], p.ld_int[sc], i - o, j - o, S);
    add_entry(p.Ci[sc], p.ld_int[sc], i - o, j - o, C);
  }
}

template <typename R, typename M>
void launch_regular(const AsmParams<M>& p, int t1_begin, int t1_end, hipStream_t st) {
  for (int t0 = t1_begin; t0 < t1_end; t0 += 65535) {
    const int rows = std::min(65535, t1_end - t0);
    // only trial blocks that reach beyond t0 can hold pairs with t2 > t1
    dim3 grid((p.F + 255) / 256, rows);
    hipLaunchKernelGGL((k_regular<R, M>), grid, dim3(256), 0, st, p, t0);
  }
}

template <typename M>
void launch_singular(const AsmParams<M>& p, const SingParams& s, hipStream_t st) {
  if (s.npairs == 0) return;
  const int per_block = 256 / WAVE;
  const int64_t blocks = (s.npairs + per_block - 1) / per_block;
  hipLaunchKernelGGL((k_singular<M>), dim3(unsigned(blocks)), dim3(256), 0, st, p, s);
}

template void launch_regular<double, double>(const AsmParams<double>&, int, int, hipStream_t);
template void launch_regular<float, float>(const AsmParams<float>&, int, int, hipStream_t);
template void launch_singular<double>(const AsmParams<double>&, const SingParams&, hipStream_t);
template void launch_singular<float>(const AsmParams<float>&, const SingParams&, hipStream_t);

}  // namespace pmchwt
