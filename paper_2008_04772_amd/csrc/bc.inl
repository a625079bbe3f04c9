// Barycentric-mesh kernels: near-field Buffa-Christiansen operators of the
// preconditioner, mixed mass and Gram matrices, incident-field projections.
//
// BC operators (Section 3.2 discretisation of P, near-field cutoff of
// Section 3.3).  A BC function lives on the dual cells of the two end points
// of its edge, and on every barycentric child of a cell it is an RT0 field
// alpha x - w.  The barycentric children are partitioned by dual cell, so the
// Galerkin entry (i, j) is the sum over the four cell pairs (end point of i,
// end point of j) and every barycentric triangle pair belongs to exactly one
// cell pair.  One wavefront takes one cell pair: it integrates all child pairs
// once (moments in LDS), contracts them against the coefficients of every
// BC function of the two cells, and adds the kept entries to the CSR values.
#include "common.hpp"
#include "kernels.hpp"

namespace pmchwt {

constexpr int BC_MAX_RING = 32;      // 2 N_v <= 32 (vertex valence <= 16)
constexpr int BC_CHUNK_PAIRS = 48;   // child pairs whose moments sit in LDS at once
constexpr int MOM_D = sizeof(Moments<double>) / sizeof(double);  // 28

struct SmallGeom {
  double P[3][3];
  int vid[3];
  double cen[3], diam2, area;
};

__device__ __forceinline__ void load_child(const CellParams& c, int ch, SmallGeom& g) {
  for (int k = 0; k < 3; ++k) {
    for (int d = 0; d < 3; ++d) g.P[k][d] = c.child_v[9 * int64_t(ch) + 3 * k + d];
    g.vid[k] = c.child_vid[3 * int64_t(ch) + k];
  }
  for (int d = 0; d < 3; ++d) g.cen[d] = c.child_cen[3 * int64_t(ch) + d];
  g.diam2 = c.child_diam2[ch];
  g.area = c.child_area[ch];
}

// Moments of one (test, trial) triangle pair, origin = test centroid.
// Identical / shared-edge / shared-vertex pairs use the Sauter-Schwab tables,
// disjoint pairs the tensor rule of their distance class.
__device__ void pair_moments(const SmallGeom& a, const SmallGeom& b, const double* const* tab,
                             const int* npts, int qn, int qm, int qf, int nk, const double* kr,
                             const double* ki, bool withC, Moments<double>* out) {
  for (int k = 0; k < nk; ++k) out[k].zero();
  double P1[3][3], P2[3][3];
  for (int v = 0; v < 3; ++v)
    for (int d = 0; d < 3; ++d) {
      P1[v][d] = a.P[v][d] - a.cen[d];
      P2[v][d] = b.P[v][d] - a.cen[d];
    }
  int oa[3], ob[3], nc = 0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      if (a.vid[i] == b.vid[j]) {
        oa[nc] = i;
        ob[nc] = j;
        ++nc;
      }
  if (nc > 0) {
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
    const double* T = tab[nc];
    const int n = npts[nc];
    const double AA = 4.0 * a.area * b.area;
    for (int q = 0; q < n; ++q) {
      const double x1 = T[5 * q], x2 = T[5 * q + 1], y1 = T[5 * q + 2], y2 = T[5 * q + 3];
      const double w = T[5 * q + 4] * AA;
      double x[3], y[3];
      for (int d = 0; d < 3; ++d) {
        x[d] = P1[oa[0]][d] + x1 * (P1[oa[1]][d] - P1[oa[0]][d]) + x2 * (P1[oa[2]][d] - P1[oa[1]][d]);
        y[d] = P2[ob[0]][d] + y1 * (P2[ob[1]][d] - P2[ob[0]][d]) + y2 * (P2[ob[2]][d] - P2[ob[1]][d]);
      }
      const double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
      const double r2 = dx * dx + dy * dy + dz * dz;
      for (int k = 0; k < nk; ++k) {
        KernelVal<double> kv = helmholtz<double>(r2, kr[k], ki[k], ki[k] != 0.0, w);
        out[k].add(kv, x, y, withC);
      }
    }
    return;
  }
  const int cls = classify_pair(a.cen, b.cen, a.diam2, b.diam2);
  const int q = cls == 0 ? qn : (cls == 1 ? qm : qf);
  const int off = c_rule_off[q], n = c_rule_n[q];
  const double AA = a.area * b.area;
  for (int i = 0; i < n; ++i) {
    double x[3];
    for (int d = 0; d < 3; ++d)
      x[d] = c_rule_l[off + i][0] * P1[0][d] + c_rule_l[off + i][1] * P1[1][d] + c_rule_l[off + i][2] * P1[2][d];
    for (int j = 0; j < n; ++j) {
      double y[3];
      for (int d = 0; d < 3; ++d)
        y[d] = c_rule_l[off + j][0] * P2[0][d] + c_rule_l[off + j][1] * P2[1][d] + c_rule_l[off + j][2] * P2[2][d];
      const double w = c_rule_w[off + i] * c_rule_w[off + j] * AA;
      const double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
      const double r2 = dx * dx + dy * dy + dz * dz;
      for (int k = 0; k < nk; ++k) {
        KernelVal<double> kv = helmholtz<double>(r2, kr[k], ki[k], ki[k] != 0.0, w);
        out[k].add(kv, x, y, withC);
      }
    }
  }
}

__global__ __launch_bounds__(64) void k_bc_nearfield(CellParams c, BCJob j) {
  __shared__ double s_mom[BC_CHUNK_PAIRS * 2 * MOM_D];
  __shared__ double s_org[BC_MAX_RING][3];
  __shared__ double s_acc[BC_MAX_RING * BC_MAX_RING / 4][8];
  const int lane = threadIdx.x;
  const int64_t pr = blockIdx.x;
  const int v = j.cpairs[2 * pr], w = j.cpairs[2 * pr + 1];
  const int b1 = c.cell_ptr[v], n1 = c.cell_ptr[v + 1] - b1;
  const int b2 = c.cell_ptr[w], n2 = c.cell_ptr[w + 1] - b2;
  const int N1 = n1 / 2, N2 = n2 / 2, nslot = N1 * N2;
  const int sc1 = c.cell_scat[v], sc2 = c.cell_scat[w];
  const bool do_int = j.want_int && sc1 == sc2;
  const bool do_ext = j.want_ext;
  int nk = 0;
  double kr[2], ki[2];
  if (do_int) {
    kr[nk] = j.k_int[2 * sc1];
    ki[nk] = j.k_int[2 * sc1 + 1];
    ++nk;
  }
  if (do_ext) {
    kr[nk] = j.k_ext;
    ki[nk] = 0.0;
    ++nk;
  }
  const bool withC = j.want_C;
  for (int s = lane; s < nslot; s += 64)
    for (int q = 0; q < 8; ++q) s_acc[s][q] = 0.0;
  const int rows_per_chunk = max(1, BC_CHUNK_PAIRS / n2);
  const double* cv = c.coef + 4 * c.coef_ptr[v];
  const double* cw = c.coef + 4 * c.coef_ptr[w];
  for (int r0 = 0; r0 < n1; r0 += rows_per_chunk) {
    const int nr = min(rows_per_chunk, n1 - r0);
    const int np = nr * n2;
    __syncthreads();
    for (int p = lane; p < np; p += 64) {
      const int u1 = r0 + p / n2, u2 = p % n2;
      SmallGeom ga, gb;
      load_child(c, c.ring[b1 + u1], ga);
      load_child(c, c.ring[b2 + u2], gb);
      Moments<double> m[2];
      pair_moments(ga, gb, j.tab, j.npts, j.q_near, j.q_medium, j.q_far, nk, kr, ki, withC, m);
      for (int k = 0; k < nk; ++k) {
        const double* f = reinterpret_cast<const double*>(&m[k]);
        for (int q = 0; q < MOM_D; ++q) s_mom[(p * 2 + k) * MOM_D + q] = f[q];
      }
      if (p % n2 == 0)
        for (int d = 0; d < 3; ++d) s_org[u1 - r0][d] = ga.cen[d];
    }
    __syncthreads();
    for (int s = lane; s < nslot; s += 64) {
      const int si = s / N2, sj = s % N2;
      double acc[8];
      for (int q = 0; q < 8; ++q) acc[q] = s_acc[s][q];
      for (int p = 0; p < np; ++p) {
        const int u1 = r0 + p / n2, u2 = p % n2;
        const double* c1 = cv + 4 * (int64_t(si) * n1 + u1);
        const double* c2 = cw + 4 * (int64_t(sj) * n2 + u2);
        const double a1 = c1[0], a2 = c2[0];
        if (a1 == 0.0 && c1[1] == 0.0 && c1[2] == 0.0 && c1[3] == 0.0) continue;
        if (a2 == 0.0 && c2[1] == 0.0 && c2[2] == 0.0 && c2[3] == 0.0) continue;
        const double* o = s_org[u1 - r0];
        // shift the fields to the pair's origin: alpha x - w = alpha x' - (w - alpha o)
        double w1[3], w2[3];
        for (int d = 0; d < 3; ++d) {
          w1[d] = c1[1 + d] - a1 * o[d];
          w2[d] = c2[1 + d] - a2 * o[d];
        }
        for (int k = 0; k < nk; ++k) {
          const Moments<double>& m = *reinterpret_cast<const Moments<double>*>(&s_mom[(p * 2 + k) * MOM_D]);
          cplx<double> S, C;
          contract<double, double>(m, a1, w1, a2, w2, kr[k], ki[k], withC, S, C);
          const int slot = (do_int && k == 0) ? 0 : 4;
          acc[slot + 0] += S.re;
          acc[slot + 1] += S.im;
          acc[slot + 2] += C.re;
          acc[slot + 3] += C.im;
        }
      }
      for (int q = 0; q < 8; ++q) s_acc[s][q] = acc[q];
    }
  }
  __syncthreads();
  const int64_t* pos = j.slot_pos + j.slot_off[pr];
  for (int s = lane; s < nslot; s += 64) {
    const int64_t ps = pos[s];
    if (ps < 0) continue;
    if (do_int) {
      atomic_add(&j.out_Si[2 * ps], s_acc[s][0]);
      atomic_add(&j.out_Si[2 * ps + 1], s_acc[s][1]);
      if (withC) {
        atomic_add(&j.out_Ci[2 * ps], s_acc[s][2]);
        atomic_add(&j.out_Ci[2 * ps + 1], s_acc[s][3]);
      }
    }
    if (do_ext) {
      atomic_add(&j.out_Se[2 * ps], s_acc[s][4]);
      atomic_add(&j.out_Se[2 * ps + 1], s_acc[s][5]);
      if (withC) {
        atomic_add(&j.out_Ce[2 * ps], s_acc[s][6]);
        atomic_add(&j.out_Ce[2 * ps + 1], s_acc[s][7]);
      }
    }
  }
}

void launch_bc_nearfield(const AsmParams<double>& geo, const CellParams& c, const BCJob& j, hipStream_t st) {
  (void)geo;
  for (int64_t p0 = 0; p0 < j.npairs; p0 += (int64_t(1) << 30)) {
    BCJob jj = j;
    jj.npairs = std::min<int64_t>(j.npairs - p0, int64_t(1) << 30);
    jj.cpairs = j.cpairs + 2 * p0;
    jj.slot_off = j.slot_off + p0;
    hipLaunchKernelGGL(k_bc_nearfield, dim3(unsigned(jj.npairs)), dim3(64), 0, st, c, jj);
  }
}

// ---------------------------------------------------------------------------
// Mixed mass matrix (M_A)_ij = int bc_j . (n x rwg_i) (Section 3.2).  One
// thread per (barycentric child, RWG local basis of its parent); the product
// of two linear fields is integrated exactly by the degree-2 rule.
// ---------------------------------------------------------------------------
__global__ void k_mass(AsmParams<double> g, CellParams c, MassJob j) {
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (tid >= int64_t(j.nchild) * 3) return;
  const int ch = int(tid / 3), a = int(tid % 3);
  const int T = j.child_parent[ch];
  const int F = g.F;
  double P[3][3];
  for (int k = 0; k < 3; ++k)
    for (int d = 0; d < 3; ++d) P[k][d] = g.tv[(3 * k + d) * F + T];
  double u[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
  double v[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
  double n[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
  const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  for (int d = 0; d < 3; ++d) n[d] /= nn;
  const double A = g.tarea[T];
  const double ar = g.tsgn[a * F + T] / (2.0 * A);
  double wr[3];
  for (int d = 0; d < 3; ++d) wr[d] = ar * P[a][d];
  const int i = g.t2e[a * F + T];
  const int sc = g.tscat[T];
  const int il = i - j.edge_off[sc];
  const int cell = j.child_cell[ch], pos = j.child_pos[ch];
  const int n2 = c.cell_ptr[cell + 1] - c.cell_ptr[cell];
  const int N = n2 / 2;
  double X[3][3];
  for (int k = 0; k < 3; ++k)
    for (int d = 0; d < 3; ++d) X[k][d] = c.child_v[9 * int64_t(ch) + 3 * k + d];
  const double Ac = c.child_area[ch];
  // degree-2 rule: interior points (2/3, 1/6, 1/6), weights 1/3
  double xq[3][3];
  for (int q = 0; q < 3; ++q)
    for (int d = 0; d < 3; ++d) {
      double l0 = (q == 0) ? 2.0 / 3.0 : 1.0 / 6.0, l1 = (q == 1) ? 2.0 / 3.0 : 1.0 / 6.0,
             l2 = (q == 2) ? 2.0 / 3.0 : 1.0 / 6.0;
      xq[q][d] = l0 * X[0][d] + l1 * X[1][d] + l2 * X[2][d];
    }
  double* out = j.out + j.mat_off[sc];
  const int64_t ld = j.ld[sc];
  for (int s = 0; s < N; ++s) {
    const double* cf = c.coef + 4 * (c.coef_ptr[cell] + int64_t(s) * n2 + pos);
    const int jj = j.inc_edges[j.inc_ptr[cell] + s] - j.edge_off[sc];
    double acc = 0.0;
    for (int q = 0; q < 3; ++q) {
      double b[3], r[3];
      for (int d = 0; d < 3; ++d) {
        b[d] = cf[0] * xq[q][d] - cf[1 + d];
        r[d] = ar * xq[q][d] - wr[d];
      }
      double nr[3] = {n[1] * r[2] - n[2] * r[1], n[2] * r[0] - n[0] * r[2], n[0] * r[1] - n[1] * r[0]};
      acc += (b[0] * nr[0] + b[1] * nr[1] + b[2] * nr[2]) / 3.0;
    }
    atomic_add(&out[int64_t(il) * ld + jj], acc * Ac);
  }
}

void launch_mass(const AsmParams<double>& geo, const CellParams& c, const MassJob& j, hipStream_t st) {
  const int64_t n = int64_t(j.nchild) * 3;
  hipLaunchKernelGGL(k_mass, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, geo, c, j);
}

// RWG Gram matrix int rwg_i . rwg_j: one thread per (triangle, a, b).
__global__ void k_gram(AsmParams<double> g, MassJob j) {
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (tid >= int64_t(g.F) * 9) return;
  const int T = int(tid / 9), a = int(tid % 9) / 3, b = int(tid % 3);
  const int F = g.F;
  double P[3][3];
  for (int k = 0; k < 3; ++k)
    for (int d = 0; d < 3; ++d) P[k][d] = g.tv[(3 * k + d) * F + T];
  const double A = g.tarea[T];
  const double sa = g.tsgn[a * F + T] / (2.0 * A), sb = g.tsgn[b * F + T] / (2.0 * A);
  double acc = 0.0;
  for (int q = 0; q < 3; ++q) {
    double x[3];
    for (int d = 0; d < 3; ++d) {
      double l0 = (q == 0) ? 2.0 / 3.0 : 1.0 / 6.0, l1 = (q == 1) ? 2.0 / 3.0 : 1.0 / 6.0,
             l2 = (q == 2) ? 2.0 / 3.0 : 1.0 / 6.0;
      x[d] = l0 * P[0][d] + l1 * P[1][d] + l2 * P[2][d];
    }
    double dot = 0.0;
    for (int d = 0; d < 3; ++d) dot += (x[d] - P[a][d]) * (x[d] - P[b][d]);
    acc += dot / 3.0;
  }
  const int sc = g.tscat[T];
  const int i = g.t2e[a * F + T] - j.edge_off[sc], jj = g.t2e[b * F + T] - j.edge_off[sc];
  atomic_add(&j.out[j.mat_off[sc] + int64_t(i) * j.ld[sc] + jj], acc * A * sa * sb);
}

void launch_gram(const AsmParams<double>& geo, const MassJob& j, hipStream_t st) {
  const int64_t n = int64_t(geo.F) * 9;
  hipLaunchKernelGGL(k_gram, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, geo, j);
}

// ---------------------------------------------------------------------------
// Incident-field projections for the right-hand side (Section 3.2):
//   g = int u^inc . (n x rwg),  h = int u^inc . rwg,
//   u^inc = [E x n ; k_e ((d x p) exp(i k_e d.x)) x n],  E = p exp(i k_e d.x),
// degree-4 six-point rule per triangle.  One thread per (triangle, wave).
// ---------------------------------------------------------------------------
__global__ void k_rhs(AsmParams<double> g, RhsJob j) {
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (tid >= int64_t(g.F) * j.nrhs) return;
  const int T = int(tid % g.F), r = int(tid / g.F);
  const int F = g.F;
  double P[3][3];
  for (int k = 0; k < 3; ++k)
    for (int d = 0; d < 3; ++d) P[k][d] = g.tv[(3 * k + d) * F + T];
  double u[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
  double v[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
  double n[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
  const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  for (int d = 0; d < 3; ++d) n[d] /= nn;
  const double A = g.tarea[T];
  const double* dr = j.dirs + 3 * r;
  const double* pl = j.pols + 6 * r;
  double pre[3], pim[3];
  for (int d = 0; d < 3; ++d) {
    pre[d] = pl[2 * d];
    pim[d] = pl[2 * d + 1];
  }
  // q = d x p
  double qre[3] = {dr[1] * pre[2] - dr[2] * pre[1], dr[2] * pre[0] - dr[0] * pre[2], dr[0] * pre[1] - dr[1] * pre[0]};
  double qim[3] = {dr[1] * pim[2] - dr[2] * pim[1], dr[2] * pim[0] - dr[0] * pim[2], dr[0] * pim[1] - dr[1] * pim[0]};
  double acc[3][8];
  for (int a = 0; a < 3; ++a)
    for (int q = 0; q < 8; ++q) acc[a][q] = 0.0;
  const int off = c_rule_off[4], nq = c_rule_n[4];
  for (int qi = 0; qi < nq; ++qi) {
    double x[3];
    for (int d = 0; d < 3; ++d)
      x[d] = c_rule_l[off + qi][0] * P[0][d] + c_rule_l[off + qi][1] * P[1][d] + c_rule_l[off + qi][2] * P[2][d];
    const double ph = j.k_ext * (dr[0] * x[0] + dr[1] * x[1] + dr[2] * x[2]);
    double sn, cs;
    sincos(ph, &sn, &cs);
    const double wq = c_rule_w[off + qi] * A;
    // E = p e, H' = k (d x p) e ; uD = E x n ; uN = H' x n
    double Ere[3], Eim[3], Hre[3], Him[3];
    for (int d = 0; d < 3; ++d) {
      Ere[d] = pre[d] * cs - pim[d] * sn;
      Eim[d] = pre[d] * sn + pim[d] * cs;
      Hre[d] = j.k_ext * (qre[d] * cs - qim[d] * sn);
      Him[d] = j.k_ext * (qre[d] * sn + qim[d] * cs);
    }
    auto crossn = [&](const double* a, double* o) {
      o[0] = a[1] * n[2] - a[2] * n[1];
      o[1] = a[2] * n[0] - a[0] * n[2];
      o[2] = a[0] * n[1] - a[1] * n[0];
    };
    double uDr[3], uDi[3], uNr[3], uNi[3];
    crossn(Ere, uDr);
    crossn(Eim, uDi);
    crossn(Hre, uNr);
    crossn(Him, uNi);
    for (int a = 0; a < 3; ++a) {
      const double s = g.tsgn[a * F + T] / (2.0 * A);
      double f[3];
      for (int d = 0; d < 3; ++d) f[d] = s * (x[d] - P[a][d]);
      double nf[3] = {n[1] * f[2] - n[2] * f[1], n[2] * f[0] - n[0] * f[2], n[0] * f[1] - n[1] * f[0]};
      double gDr = 0, gDi = 0, gNr = 0, gNi = 0, hDr = 0, hDi = 0, hNr = 0, hNi = 0;
      for (int d = 0; d < 3; ++d) {
        gDr += uDr[d] * nf[d];
        gDi += uDi[d] * nf[d];
        gNr += uNr[d] * nf[d];
        gNi += uNi[d] * nf[d];
        hDr += uDr[d] * f[d];
        hDi += uDi[d] * f[d];
        hNr += uNr[d] * f[d];
        hNi += uNi[d] * f[d];
      }
      acc[a][0] += wq * gDr;
      acc[a][1] += wq * gDi;
      acc[a][2] += wq * gNr;
      acc[a][3] += wq * gNi;
      acc[a][4] += wq * hDr;
      acc[a][5] += wq * hDi;
      acc[a][6] += wq * hNr;
      acc[a][7] += wq * hNi;
    }
  }
  for (int a = 0; a < 3; ++a) {
    const int e = g.t2e[a * F + T];
    double* gD = j.g + 2 * ((int64_t(r) * 2 + 0) * j.E_tot + e);
    double* gN = j.g + 2 * ((int64_t(r) * 2 + 1) * j.E_tot + e);
    double* hD = j.h + 2 * ((int64_t(r) * 2 + 0) * j.E_tot + e);
    double* hN = j.h + 2 * ((int64_t(r) * 2 + 1) * j.E_tot + e);
    atomic_add(gD, acc[a][0]);
    atomic_add(gD + 1, acc[a][1]);
    atomic_add(gN, acc[a][2]);
    atomic_add(gN + 1, acc[a][3]);
    atomic_add(hD, acc[a][4]);
    atomic_add(hD + 1, acc[a][5]);
    atomic_add(hN, acc[a][6]);
    atomic_add(hN + 1, acc[a][7]);
  }
}

void launch_rhs(const AsmParams<double>& geo, const RhsJob& j, hipStream_t st) {
  const int64_t n = int64_t(geo.F) * j.nrhs;
  hipLaunchKernelGGL(k_rhs, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, geo, j);
}

// ---------------------------------------------------------------------------
// Far field (Stratton-Chu exterior representation, Section 2):
//   F(xh) = -(i/4pi) [k xh x V_D + V_N - xh (xh . V_N)],
//   V = int u(y) exp(-i k xh . y) ds(y)   (degree-4 rule per triangle).
// Vectors x are [rhs][D (E_tot) ; N (E_tot)] complex128.  One thread per
// (direction, wave), looping over the triangles.
// ---------------------------------------------------------------------------
__global__ void k_far(AsmParams<double> g, const double* x, int64_t E_tot, int nrhs, double k,
                      const double* obs, int nobs, double* Fout) {
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (tid >= int64_t(nobs) * nrhs) return;
  const int o = int(tid % nobs), r = int(tid / nobs);
  const double xh[3] = {obs[3 * o], obs[3 * o + 1], obs[3 * o + 2]};
  const double* xD = x + 2 * (int64_t(r) * 2 * E_tot);
  const double* xN = xD + 2 * E_tot;
  double VD[6] = {0, 0, 0, 0, 0, 0}, VN[6] = {0, 0, 0, 0, 0, 0};
  const int F = g.F;
  const int off = c_rule_off[4], nq = c_rule_n[4];
  for (int T = 0; T < F; ++T) {
    double P[3][3];
    for (int kk = 0; kk < 3; ++kk)
      for (int d = 0; d < 3; ++d) P[kk][d] = g.tv[(3 * kk + d) * F + T];
    const double A = g.tarea[T];
    double cD[3][2], cN[3][2], s[3];
    for (int a = 0; a < 3; ++a) {
      const int e = g.t2e[a * F + T];
      s[a] = g.tsgn[a * F + T] / (2.0 * A);
      cD[a][0] = xD[2 * e];
      cD[a][1] = xD[2 * e + 1];
      cN[a][0] = xN[2 * e];
      cN[a][1] = xN[2 * e + 1];
    }
    for (int q = 0; q < nq; ++q) {
      double y[3];
      for (int d = 0; d < 3; ++d)
        y[d] = c_rule_l[off + q][0] * P[0][d] + c_rule_l[off + q][1] * P[1][d] + c_rule_l[off + q][2] * P[2][d];
      double sn, cs;
      sincos(-k * (xh[0] * y[0] + xh[1] * y[1] + xh[2] * y[2]), &sn, &cs);
      const double wq = c_rule_w[off + q] * A;
      const double er = wq * cs, ei = wq * sn;
      for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 3; ++d) {
          const double f = s[a] * (y[d] - P[a][d]);
          // (cD f) * e
          VD[2 * d] += f * (cD[a][0] * er - cD[a][1] * ei);
          VD[2 * d + 1] += f * (cD[a][0] * ei + cD[a][1] * er);
          VN[2 * d] += f * (cN[a][0] * er - cN[a][1] * ei);
          VN[2 * d + 1] += f * (cN[a][0] * ei + cN[a][1] * er);
        }
    }
  }
  // B = k xh x VD + VN - xh (xh . VN);  F = -(i/4pi) B
  double xv_re = xh[0] * VN[0] + xh[1] * VN[2] + xh[2] * VN[4];
  double xv_im = xh[0] * VN[1] + xh[1] * VN[3] + xh[2] * VN[5];
  double B[6];
  for (int d = 0; d < 3; ++d) {
    const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
    const double cr = xh[d1] * VD[2 * d2] - xh[d2] * VD[2 * d1];
    const double ci = xh[d1] * VD[2 * d2 + 1] - xh[d2] * VD[2 * d1 + 1];
    B[2 * d] = k * cr + VN[2 * d] - xh[d] * xv_re;
    B[2 * d + 1] = k * ci + VN[2 * d + 1] - xh[d] * xv_im;
  }
  double* out = Fout + 6 * (int64_t(r) * nobs + o);
  for (int d = 0; d < 3; ++d) {
    // -(i/4pi)(b_re + i b_im) = (b_im - i b_re)/(4pi)
    out[2 * d] = B[2 * d + 1] * INV_FOUR_PI;
    out[2 * d + 1] = -B[2 * d] * INV_FOUR_PI;
  }
}

void launch_far_field(const AsmParams<double>& geo, const double* x, int64_t E_tot, int nrhs, double k,
                      const double* obs, int nobs, double* F_out, hipStream_t st) {
  const int64_t n = int64_t(nobs) * nrhs;
  hipLaunchKernelGGL(k_far, dim3(unsigned((n + 127) / 128)), dim3(128), 0, st, geo, x, E_tot, nrhs, k, obs, nobs,
                     F_out);
}

// sigma_sca[r] = sum_o w_o |F_o|^2
__global__ void k_sigma_sca(const double* F, int nobs, const double* w, double* out) {
  __shared__ double red[256];
  const int r = blockIdx.x;
  double acc = 0.0;
  for (int o = threadIdx.x; o < nobs; o += blockDim.x) {
    const double* f = F + 6 * (int64_t(r) * nobs + o);
    double s = 0.0;
    for (int q = 0; q < 6; ++q) s += f[q] * f[q];
    acc += w[o] * s;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[r] = red[0];
}

void launch_sigma_sca(const double* F, int nobs, int nrhs, const double* w, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sigma_sca, dim3(nrhs), dim3(256), 0, st, F, nobs, w, out);
}

}  // namespace pmchwt
