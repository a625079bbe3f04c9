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

__device__ __forceinline__ SmallGeom load_child(const CellParams& c, int ch) {
  SmallGeom g;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int d = 0; d < 3; ++d) g.P[k][d] = c.child_v[9 * int64_t(ch) + 3 * k + d];
    g.vid[k] = c.child_vid[3 * int64_t(ch) + k];
  }
  for (int d = 0; d < 3; ++d) g.cen[d] = c.child_cen[3 * int64_t(ch) + d];
  g.diam2 = c.child_diam2[ch];
  g.area = c.child_area[ch];
  return g;
}

// Moments of one (test, trial) triangle pair at one wavenumber, origin = test
// centroid, accumulated in precision R (coordinates are made relative to the
// test centroid in FP64 first).  Identical / shared-edge / shared-vertex pairs
// use the Sauter-Schwab tables (tab1..tab3 with n1..n3 records), disjoint
// pairs the tensor rule of their distance class (classified in FP64).
template <typename R>
__device__ __forceinline__ void pair_moments(const SmallGeom a, const SmallGeom b, const double* tab1,
                                             const double* tab2, const double* tab3, int n1, int n2, int n3, int qn,
                                             int qm, int qf, R kr, R ki, bool withC, Moments<R>& out) {
  out.zero();
  R P1[3][3], P2[3][3];
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      P1[v][d] = R(a.P[v][d] - a.cen[d]);
      P2[v][d] = R(b.P[v][d] - a.cen[d]);
    }
  const bool decay = ki != R(0);
  int oa, ob;
  const int nc = shared_order(a.vid, b.vid, oa, ob);
  if (nc > 0) {
    R Q1[3][3], Q2[3][3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      const int ia = (oa >> (2 * v)) & 3, ib = (ob >> (2 * v)) & 3;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const R c1[3] = {P1[0][d], P1[1][d], P1[2][d]}, c2[3] = {P2[0][d], P2[1][d], P2[2][d]};
        Q1[v][d] = pick3(c1, ia);
        Q2[v][d] = pick3(c2, ib);
      }
    }
    const double* T = nc == 1 ? tab1 : (nc == 2 ? tab2 : tab3);
    const int n = nc == 1 ? n1 : (nc == 2 ? n2 : n3);
    const R AA = R(4.0 * a.area * b.area);
    for (int q = 0; q < n; ++q) {
      const R x1 = R(T[5 * q]), x2 = R(T[5 * q + 1]), y1 = R(T[5 * q + 2]), y2 = R(T[5 * q + 3]);
      const R w = R(T[5 * q + 4]) * AA;
      R x[3], y[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        x[d] = Q1[0][d] + x1 * (Q1[1][d] - Q1[0][d]) + x2 * (Q1[2][d] - Q1[1][d]);
        y[d] = Q2[0][d] + y1 * (Q2[1][d] - Q2[0][d]) + y2 * (Q2[2][d] - Q2[1][d]);
      }
      const R dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
      const R r2 = dx * dx + dy * dy + dz * dz;
      out.add(helmholtz<R>(r2, kr, ki, decay, w), x, y, withC);
    }
    return;
  }
  const int cls = classify_pair(a.cen[0], a.cen[1], a.cen[2], b.cen[0], b.cen[1], b.cen[2], a.diam2, b.diam2);
  const int q = cls == 0 ? qn : (cls == 1 ? qm : qf);
  const int off = c_rule_off[q], n = c_rule_n[q];
  const R AA = R(a.area * b.area);
  for (int i = 0; i < n; ++i) {
    R x[3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
      x[d] = R(c_rule_l[off + i][0]) * P1[0][d] + R(c_rule_l[off + i][1]) * P1[1][d] +
             R(c_rule_l[off + i][2]) * P1[2][d];
    for (int jq = 0; jq < n; ++jq) {
      R y[3];
#pragma unroll
      for (int d = 0; d < 3; ++d)
        y[d] = R(c_rule_l[off + jq][0]) * P2[0][d] + R(c_rule_l[off + jq][1]) * P2[1][d] +
               R(c_rule_l[off + jq][2]) * P2[2][d];
      const R w = R(c_rule_w[off + i] * c_rule_w[off + jq]) * AA;
      const R dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
      const R r2 = dx * dx + dy * dy + dz * dz;
      out.add(helmholtz<R>(r2, kr, ki, decay, w), x, y, withC);
    }
  }
}

// Half contraction over the trial side for one (test child u1, trial
// function slot sj): with u = a1 x - w1, v = a2 y - w2 (pair origin),
//   Sv = a1 Ta + w1 . Tb,  Sd = a1 Td,  C = a1 Tc + w1 . Te,
//   Ta = sum (a2 Mxy - w2 . Mx),  Tb = sum (w2 M0 - a2 My),  Td = sum 4 a2 M0,
//   Tc = -sum w2 . Nx,            Te = sum (a2 Nx - Nd x w2),
// sums over the trial children u2 of the cell.
template <typename R>
struct HalfC {
  R v[18];  // Ta(2) Tb(6) Td(2) Tc(2) Te(6)
};

// R: precision of the pair moments and contractions (FP64, or FP32 for a
// mixed-precision preconditioner); the kept entries are added in FP64.
// NK: wavenumbers the LDS holds per child pair (1 or 2, the most any cell
// pair of the launch needs); the slot sums stay in registers, slots lane,
// lane + 64, ... of the N_v x N_w <= 256 of the pair
constexpr int BC_SLOTS_PER_LANE = BC_MAX_RING * BC_MAX_RING / 4 / 64;
template <typename R, int NK>
__global__ __launch_bounds__(64) void k_bc_nearfield(CellParams c, BCJob j) {
  __shared__ R s_mom[BC_CHUNK_PAIRS * NK * MOM_D];
  __shared__ double s_org[BC_MAX_RING][3];
  __shared__ HalfC<R> s_half[BC_CHUNK_PAIRS / 2][NK];
  const int lane = threadIdx.x;
  const int64_t pr = blockIdx.x;
  const int v = j.cpairs[2 * pr], w = j.cpairs[2 * pr + 1];
  const int b1 = c.cell_ptr[v], n1 = c.cell_ptr[v + 1] - b1;
  const int b2 = c.cell_ptr[w], n2 = c.cell_ptr[w + 1] - b2;
  const int N1 = n1 / 2, N2 = n2 / 2, nslot = N1 * N2;
  const int sc1 = c.cell_scat[v], sc2 = c.cell_scat[w];
  const bool do_int = j.want_int && sc1 == sc2;
  const bool do_ext = j.want_ext;
  // wavenumber 0 is the interior one when present, else the exterior one
  const int nk = int(do_int) + int(do_ext);
  const double kr0 = do_int ? j.k_int[2 * sc1] : j.k_ext, ki0 = do_int ? j.k_int[2 * sc1 + 1] : 0.0;
  const double kr1 = j.k_ext, ki1 = 0.0;
  const bool withC = j.want_C;
  R acc[BC_SLOTS_PER_LANE][8];
#pragma unroll
  for (int t = 0; t < BC_SLOTS_PER_LANE; ++t)
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[t][q] = R(0);
  const int rows_per_chunk = max(1, BC_CHUNK_PAIRS / n2);
  const double* cv = c.coef + 4 * c.coef_ptr[v];
  const double* cw = c.coef + 4 * c.coef_ptr[w];
  for (int r0 = 0; r0 < n1; r0 += rows_per_chunk) {
    const int nr = min(rows_per_chunk, n1 - r0);
    const int np = nr * n2;
    __syncthreads();
    // ---- A: moments of every child pair of this chunk
    for (int p = lane; p < np; p += 64) {
      const int u1 = r0 + p / n2, u2 = p % n2;
      const SmallGeom ga = load_child(c, c.ring[b1 + u1]);
      const SmallGeom gb = load_child(c, c.ring[b2 + u2]);
      for (int k = 0; k < nk; ++k) {
        Moments<R> m;
        pair_moments<R>(ga, gb, j.tab[1], j.tab[2], j.tab[3], j.npts[1], j.npts[2], j.npts[3], j.q_near, j.q_medium,
                        j.q_far, R(k == 0 ? kr0 : kr1), R(k == 0 ? ki0 : ki1), withC, m);
        const R* f = reinterpret_cast<const R*>(&m);
#pragma unroll
        for (int q = 0; q < MOM_D; ++q) s_mom[(p * NK + k) * MOM_D + q] = f[q];
      }
      if (u2 == 0)
        for (int d = 0; d < 3; ++d) s_org[u1 - r0][d] = ga.cen[d];
    }
    __syncthreads();
    // ---- B1: half contraction over the trial children, one (u1, sj) per lane
    const int nh = nr * N2;
    for (int hq = lane; hq < nh; hq += 64) {
      const int ur = hq / N2, sj = hq % N2;
      const double* o = s_org[ur];
      for (int k = 0; k < nk; ++k) {
        R T[18];
#pragma unroll
        for (int q = 0; q < 18; ++q) T[q] = R(0);
        for (int u2 = 0; u2 < n2; ++u2) {
          const double* c2 = cw + 4 * (int64_t(sj) * n2 + u2);
          const R a2 = R(c2[0]);
          const R w2[3] = {R(c2[1] - c2[0] * o[0]), R(c2[2] - c2[0] * o[1]), R(c2[3] - c2[0] * o[2])};
          const Moments<R>& m = *reinterpret_cast<const Moments<R>*>(&s_mom[((ur * n2 + u2) * NK + k) * MOM_D]);
          // Ta
          T[0] += a2 * m.Mxy.re - (w2[0] * m.Mx[0].re + w2[1] * m.Mx[1].re + w2[2] * m.Mx[2].re);
          T[1] += a2 * m.Mxy.im - (w2[0] * m.Mx[0].im + w2[1] * m.Mx[1].im + w2[2] * m.Mx[2].im);
#pragma unroll
          for (int d = 0; d < 3; ++d) {  // Tb
            T[2 + 2 * d] += w2[d] * m.M0.re - a2 * m.My[d].re;
            T[3 + 2 * d] += w2[d] * m.M0.im - a2 * m.My[d].im;
          }
          T[8] += R(4) * a2 * m.M0.re;  // Td
          T[9] += R(4) * a2 * m.M0.im;
          if (withC) {
            T[10] -= w2[0] * m.Nx[0].re + w2[1] * m.Nx[1].re + w2[2] * m.Nx[2].re;  // Tc
            T[11] -= w2[0] * m.Nx[0].im + w2[1] * m.Nx[1].im + w2[2] * m.Nx[2].im;
#pragma unroll
            for (int d = 0; d < 3; ++d) {  // Te = a2 Nx - Nd x w2
              const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
              T[12 + 2 * d] += a2 * m.Nx[d].re - (m.Nd[d1].re * w2[d2] - m.Nd[d2].re * w2[d1]);
              T[13 + 2 * d] += a2 * m.Nx[d].im - (m.Nd[d1].im * w2[d2] - m.Nd[d2].im * w2[d1]);
            }
          }
        }
#pragma unroll
        for (int q = 0; q < 18; ++q) s_half[hq][k].v[q] = T[q];
      }
    }
    __syncthreads();
    // ---- B2: test side, one (si, sj) per lane
#pragma unroll
    for (int t = 0; t < BC_SLOTS_PER_LANE; ++t) {
      const int s = lane + 64 * t;
      if (s >= nslot) continue;
      const int si = s / N2, sj = s % N2;
      for (int k = 0; k < nk; ++k) {
        R sv_re = 0, sv_im = 0, sd_re = 0, sd_im = 0, cc_re = 0, cc_im = 0;
        for (int ur = 0; ur < nr; ++ur) {
          const double* c1 = cv + 4 * (int64_t(si) * n1 + r0 + ur);
          const R a1 = R(c1[0]);
          const double* o = s_org[ur];
          const R w1[3] = {R(c1[1] - c1[0] * o[0]), R(c1[2] - c1[0] * o[1]), R(c1[3] - c1[0] * o[2])};
          const R* T = s_half[ur * N2 + sj][k].v;
          sv_re += a1 * T[0] + w1[0] * T[2] + w1[1] * T[4] + w1[2] * T[6];
          sv_im += a1 * T[1] + w1[0] * T[3] + w1[1] * T[5] + w1[2] * T[7];
          sd_re += a1 * T[8];
          sd_im += a1 * T[9];
          if (withC) {
            cc_re += a1 * T[10] + w1[0] * T[12] + w1[1] * T[14] + w1[2] * T[16];
            cc_im += a1 * T[11] + w1[0] * T[13] + w1[1] * T[15] + w1[2] * T[17];
          }
        }
        // S = -ik Sv - Sd/(ik) = (ki - i kr) Sv + i Sd conj(k)/|k|^2
        const double krk = k == 0 ? kr0 : kr1, kik = k == 0 ? ki0 : ki1;
        const double k2 = krk * krk + kik * kik;
        const double t_re = (sd_re * krk + sd_im * kik) / k2, t_im = (sd_im * krk - sd_re * kik) / k2;
        const double v[4] = {kik * sv_re + krk * sv_im - t_im, kik * sv_im - krk * sv_re + t_re, cc_re, cc_im};
        const bool to_int = do_int && k == 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          acc[t][q] += to_int ? R(v[q]) : R(0);
          acc[t][4 + q] += to_int ? R(0) : R(v[q]);
        }
      }
    }
  }
  // every slot of a kept entry written once (zero for an operator this pair
  // does not reach); launch_bc_gather adds the four slots of each entry
  const int64_t sbase = j.slot_off[pr];
  const int64_t* pos = j.slot_pos + sbase;
  const int oi = 0, oe = j.want_int ? (withC ? 4 : 2) : 0;
#pragma unroll
  for (int t = 0; t < BC_SLOTS_PER_LANE; ++t) {
    const int s = lane + 64 * t;
    if (s >= nslot) continue;
    if (pos[s] < 0) continue;
    double* o = j.slot_val + (sbase + s) * j.nv;
    if (j.want_int) {
      o[oi] = do_int ? double(acc[t][0]) : 0.0;
      o[oi + 1] = do_int ? double(acc[t][1]) : 0.0;
      if (withC) {
        o[oi + 2] = do_int ? double(acc[t][2]) : 0.0;
        o[oi + 3] = do_int ? double(acc[t][3]) : 0.0;
      }
    }
    if (do_ext) {
      o[oe] = double(acc[t][4]);
      o[oe + 1] = double(acc[t][5]);
      if (withC) {
        o[oe + 2] = double(acc[t][6]);
        o[oe + 3] = double(acc[t][7]);
      }
    }
  }
}

// one thread per kept entry: the sum of its four slots, in the order 2a + b
__global__ void k_bc_gather(BCJob j) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= j.nnz) return;
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int q = 0; q < 4; ++q) {
    const int64_t sl = j.entry_slots[4 * p + q];
    if (sl < 0 || sl >= j.nslots) continue;  // every kept entry has its four slots; guard only
    const double* o = j.slot_val + sl * j.nv;
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if (c < j.nv) v[c] += o[c];
  }
  int c = 0;
  if (j.want_int) {
    j.out_Si[2 * p] = v[c];
    j.out_Si[2 * p + 1] = v[c + 1];
    c += 2;
    if (j.want_C) {
      j.out_Ci[2 * p] = v[c];
      j.out_Ci[2 * p + 1] = v[c + 1];
      c += 2;
    }
  }
  if (j.want_ext) {
    j.out_Se[2 * p] = v[c];
    j.out_Se[2 * p + 1] = v[c + 1];
    c += 2;
    if (j.want_C) {
      j.out_Ce[2 * p] = v[c];
      j.out_Ce[2 * p + 1] = v[c + 1];
    }
  }
}

void launch_bc_gather(const BCJob& j, hipStream_t st) {
  if (j.nnz > 0) hipLaunchKernelGGL(k_bc_gather, dim3(unsigned((j.nnz + 255) / 256)), dim3(256), 0, st, j);
}

void launch_bc_nearfield(const AsmParams<double>& geo, const CellParams& c, const BCJob& j, hipStream_t st) {
  (void)geo;
  for (int64_t p0 = 0; p0 < j.npairs; p0 += (int64_t(1) << 30)) {
    BCJob jj = j;
    jj.npairs = std::min<int64_t>(j.npairs - p0, int64_t(1) << 30);
    jj.cpairs = j.cpairs + 2 * p0;
    jj.slot_off = j.slot_off + p0;
    const bool two = j.want_int && j.want_ext;  // a cell pair may need both wavenumbers
    if (j.fp32) {
      if (two)
        hipLaunchKernelGGL((k_bc_nearfield<float, 2>), dim3(unsigned(jj.npairs)), dim3(64), 0, st, c, jj);
      else
        hipLaunchKernelGGL((k_bc_nearfield<float, 1>), dim3(unsigned(jj.npairs)), dim3(64), 0, st, c, jj);
    } else {
      if (two)
        hipLaunchKernelGGL((k_bc_nearfield<double, 2>), dim3(unsigned(jj.npairs)), dim3(64), 0, st, c, jj);
      else
        hipLaunchKernelGGL((k_bc_nearfield<double, 1>), dim3(unsigned(jj.npairs)), dim3(64), 0, st, c, jj);
    }
  }
}

// ---------------------------------------------------------------------------
// Mixed mass matrix (M_A)_ij = int bc_j . (n x rwg_i) (Section 3.2).  One
// thread per entry of M_A's structural pattern: the sum over the barycentric
// children of T+(i), then T-(i) (six each, in their order), of the children
// lying in a dual cell at an end of edge j, where bc_j is linear and the
// product of two linear fields is integrated exactly by the degree-2 rule.
// One writer per entry and a fixed order: the values do not depend on the
// schedule.  M_A^T takes the same values by a transposed gather.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t row_of(const int64_t* rowptr, int n, int64_t p) {
  int lo = 0, hi = n;  // the last row r with rowptr[r] <= p
  while (hi - lo > 1) {
    const int m = (lo + hi) >> 1;
    if (rowptr[m] <= p)
      lo = m;
    else
      hi = m;
  }
  return lo;
}

__global__ void k_mass(AsmParams<double> g, CellParams c, MassJob j) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= j.nnz_m) return;
  const int i = int(row_of(j.m_rowptr, j.E, p));
  const int sc = j.edge_scat[i];
  const int jg = j.m_col[p] + j.edge_off[sc];
  const int F = g.F;
  double sum = 0.0;
  for (int side = 0; side < 2; ++side) {
    const int slot = j.edge_slots[2 * i + side];
    const int T = slot / 3, a = slot - 3 * (slot / 3);
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
    for (int k = 0; k < 6; ++k) {
      const int ch = 6 * T + k;
      const int cell = j.child_cell[ch];
      const int i0 = j.inc_ptr[cell], N = j.inc_ptr[cell + 1] - i0;
      int s = -1;
      for (int t = 0; t < N; ++t)
        if (j.inc_edges[i0 + t] == jg) s = t;
      if (s < 0) continue;  // bc_j vanishes on this child
      const int n2 = c.cell_ptr[cell + 1] - c.cell_ptr[cell];
      const double* cf = c.coef + 4 * (c.coef_ptr[cell] + int64_t(s) * n2 + j.child_pos[ch]);
      double X[3][3];
      for (int q = 0; q < 3; ++q)
        for (int d = 0; d < 3; ++d) X[q][d] = c.child_v[9 * int64_t(ch) + 3 * q + d];
      double acc = 0.0;
      for (int q = 0; q < 3; ++q) {  // interior points (2/3, 1/6, 1/6), weights 1/3
        double b[3], r[3];
        for (int d = 0; d < 3; ++d) {
          const double l0 = (q == 0) ? 2.0 / 3.0 : 1.0 / 6.0, l1 = (q == 1) ? 2.0 / 3.0 : 1.0 / 6.0,
                       l2 = (q == 2) ? 2.0 / 3.0 : 1.0 / 6.0;
          const double xq = l0 * X[0][d] + l1 * X[1][d] + l2 * X[2][d];
          b[d] = cf[0] * xq - cf[1 + d];
          r[d] = ar * xq - wr[d];
        }
        const double nr[3] = {n[1] * r[2] - n[2] * r[1], n[2] * r[0] - n[0] * r[2], n[0] * r[1] - n[1] * r[0]};
        acc += (b[0] * nr[0] + b[1] * nr[1] + b[2] * nr[2]) / 3.0;
      }
      sum += acc * c.child_area[ch];
    }
  }
  j.m_val[p] = sum;
}

// (M_A^T)_{j i} = (M_A)_{i j}: one thread per entry, the value read from row
// i of M_A (ascending columns, binary search)
__global__ void k_mass_trans(MassJob j) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= j.nnz_t) return;
  const int jg = int(row_of(j.t_rowptr, j.E, p));
  const int sc = j.edge_scat[jg], off = j.edge_off[sc];
  const int i = j.t_col[p] + off, jl = jg - off;
  int64_t a0 = j.m_rowptr[i], a1 = j.m_rowptr[i + 1];
  const int64_t me = a1;
  while (a0 < a1) {
    const int64_t m = (a0 + a1) >> 1;
    if (j.m_col[m] < jl)
      a0 = m + 1;
    else
      a1 = m;
  }
  j.t_val[p] = (a0 < me && j.m_col[a0] == jl) ? j.m_val[a0] : 0.0;
}

constexpr int MASS_ROW_CAP = 128;  // candidate columns of one row of M_A or M_A^T

__global__ void k_mass_pattern(MassPatternJob J, int fill) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= J.E) return;
  int cand[MASS_ROW_CAP];
  int n = 0;
  bool over = false;
  const int off = J.edge_off[J.edge_scat[r]];
  if (!J.trans) {
    for (int side = 0; side < 2; ++side) {
      const int T = J.edge_slots[2 * r + side] / 3;
      for (int a = 0; a < 3; ++a) {
        const int v = J.tvid[a * J.F + T];
        for (int p = J.inc_ptr[v]; p < J.inc_ptr[v + 1]; ++p) {
          if (n < MASS_ROW_CAP)
            cand[n++] = J.inc_edges[p] - off;
          else
            over = true;
        }
      }
    }
  } else {
    for (int end = 0; end < 2; ++end) {
      const int v = J.ends[2 * r + end];
      for (int p = J.v2t_ptr[v]; p < J.v2t_ptr[v + 1]; ++p) {
        const int T = J.v2t[p];
        for (int a = 0; a < 3; ++a) {
          if (n < MASS_ROW_CAP)
            cand[n++] = J.t2e[a * J.F + T] - off;
          else
            over = true;
        }
      }
    }
  }
  for (int k = 1; k < n; ++k) {  // insertion sort
    const int v = cand[k];
    int q = k - 1;
    while (q >= 0 && cand[q] > v) {
      cand[q + 1] = cand[q];
      --q;
    }
    cand[q + 1] = v;
  }
  int m = 0;
  for (int k = 0; k < n; ++k)
    if (k == 0 || cand[k] != cand[k - 1]) cand[m++] = cand[k];
  if (!fill) {
    J.cnt[r] = m;
    atomicMax(&J.stats[0], m);
    if (over) atomicMax(&J.stats[1], 1);
    return;
  }
  const int64_t b = J.rowptr[r];
  for (int k = 0; k < m; ++k) J.col[b + k] = cand[k];
}

void launch_mass_pattern(const MassPatternJob& J, bool fill, hipStream_t st) {
  if (J.E > 0)
    hipLaunchKernelGGL(k_mass_pattern, dim3(unsigned((J.E + 127) / 128)), dim3(128), 0, st, J, fill ? 1 : 0);
}

// one thread per row: the row's entries into a zeroed dense row-major matrix
__global__ void k_csr_to_dense(const int64_t* rowptr, const int32_t* col, const double* val, int n, double* out,
                               int64_t ld) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  for (int64_t p = rowptr[r]; p < rowptr[r + 1]; ++p) out[int64_t(r) * ld + col[p]] = val[p];
}

void launch_csr_to_dense(const int64_t* rowptr, const int32_t* col, const double* val, int n, double* out,
                         int64_t ld, hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(k_csr_to_dense, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, rowptr, col, val, n, out,
                       ld);
}

// out[k] = in[k] - in[0], k <= n
__global__ void k_rebase_i64(const int64_t* in, int64_t n, int64_t* out) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k <= n) out[k] = in[k] - in[0];
}

void launch_rebase_i64(const int64_t* in, int64_t n, int64_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_rebase_i64, dim3(unsigned((n + 256) / 256)), dim3(256), 0, st, in, n, out);
}

void launch_mass(const AsmParams<double>& geo, const CellParams& c, const MassJob& j, hipStream_t st) {
  if (j.nnz_m > 0) hipLaunchKernelGGL(k_mass, dim3(unsigned((j.nnz_m + 255) / 256)), dim3(256), 0, st, geo, c, j);
  if (j.nnz_t > 0) hipLaunchKernelGGL(k_mass_trans, dim3(unsigned((j.nnz_t + 255) / 256)), dim3(256), 0, st, j);
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
  // an off-diagonal entry has one contribution, a diagonal one two (whose
  // sum does not depend on their order)
  atomic_add(&j.gram_val[j.gram_pos[tid]], acc * A * sa * sb);
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
    sincos_taylor(ph, &sn, &cs);
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
// Far field in three passes.  The currents are RT0 fields, so on every
// quadrature point y of the degree-4 rule the surface currents are known
// vectors; the pattern is then a non-uniform Fourier sum over the points.
//   pass 1: per point, y and the weighted currents w |T| (J_D, J_N)(y)
//   pass 2: per observation direction and segment of points, the partial sums
//           V = sum exp(-ik xh.y) J(y) (point tiles staged in LDS)
//   pass 3: per direction, the sum over segments and
//           F = -(i/4pi) (k xh x V_D + V_N - xh (xh.V_N)).
constexpr int FAR_TILE = 256;   // points per LDS tile
constexpr int FAR_BLOCK = 256;  // directions per workgroup

__global__ void k_far_points(AsmParams<double> g, const double* x, int64_t E_tot, int nrhs, int64_t npts,
                             double* ypts, double* J) {
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (tid >= npts) return;
  const int F = g.F;
  const int off = c_rule_off[4], nq = c_rule_n[4];
  const int T = int(tid / nq), q = int(tid % nq);
  double P[3][3];
  for (int kk = 0; kk < 3; ++kk)
    for (int d = 0; d < 3; ++d) P[kk][d] = g.tv[(3 * kk + d) * F + T];
  const double A = g.tarea[T];
  double y[3];
  for (int d = 0; d < 3; ++d)
    y[d] = c_rule_l[off + q][0] * P[0][d] + c_rule_l[off + q][1] * P[1][d] + c_rule_l[off + q][2] * P[2][d];
  for (int d = 0; d < 3; ++d) ypts[4 * tid + d] = y[d];
  ypts[4 * tid + 3] = 0.0;
  const double wq = c_rule_w[off + q] * A;
  for (int r = 0; r < nrhs; ++r) {
    const double* xD = x + 2 * (int64_t(r) * 2 * E_tot);
    const double* xN = xD + 2 * E_tot;
    double jv[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int a = 0; a < 3; ++a) {
      const int e = g.t2e[a * F + T];
      const double s = wq * g.tsgn[a * F + T] / (2.0 * A);
      for (int d = 0; d < 3; ++d) {
        const double f = s * (y[d] - P[a][d]);
        jv[2 * d] += f * xD[2 * e];
        jv[2 * d + 1] += f * xD[2 * e + 1];
        jv[6 + 2 * d] += f * xN[2 * e];
        jv[6 + 2 * d + 1] += f * xN[2 * e + 1];
      }
    }
    double* o = J + 12 * (int64_t(r) * npts + tid);
    for (int c = 0; c < 12; ++c) o[c] = jv[c];
  }
}

// grid (direction blocks, segments, rhs); partial sums at
// part[((r * nseg + s) * 12 + c) * nobs + o]
__global__ __launch_bounds__(FAR_BLOCK) void k_far_sum(const double* ypts, const double* J, int64_t npts,
                                                       int64_t seg_len, int nseg, double k, const double* obs,
                                                       int nobs, double* part) {
  __shared__ double s_y[FAR_TILE][4];
  __shared__ double s_j[FAR_TILE][12];
  const int o = blockIdx.x * FAR_BLOCK + threadIdx.x;
  const int sg = blockIdx.y, r = blockIdx.z;
  const bool live = o < nobs;
  double xh[3] = {0, 0, 0};
  if (live)
    for (int d = 0; d < 3; ++d) xh[d] = -k * obs[3 * o + d];
  double V[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int64_t p0 = int64_t(sg) * seg_len, p1 = min(npts, p0 + seg_len);
  const double* Jr = J + 12 * (int64_t(r) * npts);
  for (int64_t t0 = p0; t0 < p1; t0 += FAR_TILE) {
    const int nt = int(min<int64_t>(FAR_TILE, p1 - t0));
    __syncthreads();
    for (int i = threadIdx.x; i < nt * 4; i += FAR_BLOCK) s_y[i >> 2][i & 3] = ypts[4 * t0 + i];
    for (int i = threadIdx.x; i < nt * 12; i += FAR_BLOCK) s_j[i / 12][i % 12] = Jr[12 * t0 + i];
    __syncthreads();
    for (int t = 0; t < nt; ++t) {
      double sn, cs;
      sincos_taylor(xh[0] * s_y[t][0] + xh[1] * s_y[t][1] + xh[2] * s_y[t][2], &sn, &cs);
      for (int c = 0; c < 6; ++c) {
        const double jr = s_j[t][2 * c], ji = s_j[t][2 * c + 1];
        V[2 * c] += cs * jr - sn * ji;
        V[2 * c + 1] += cs * ji + sn * jr;
      }
    }
  }
  if (!live) return;
  double* out = part + (int64_t(r) * nseg + sg) * 12 * int64_t(nobs) + o;
  for (int c = 0; c < 12; ++c) out[int64_t(c) * nobs] = V[c];
}

// F(xh) = -(i / 4 pi) [k xh x V_D + V_N - xh (xh . V_N)] from the sums V (V_D
// then V_N, (re, im) per component) into out (3 complex)
__device__ __forceinline__ void far_from_sums(const double (&xh)[3], const double (&V)[12], double k,
                                              double* __restrict__ out) {
  const double* VD = V;
  const double* VN = V + 6;
  const double xv_re = xh[0] * VN[0] + xh[1] * VN[2] + xh[2] * VN[4];
  const double xv_im = xh[0] * VN[1] + xh[1] * VN[3] + xh[2] * VN[5];
  for (int d = 0; d < 3; ++d) {
    const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
    const double cr = xh[d1] * VD[2 * d2] - xh[d2] * VD[2 * d1];
    const double ci = xh[d1] * VD[2 * d2 + 1] - xh[d2] * VD[2 * d1 + 1];
    const double b_re = k * cr + VN[2 * d] - xh[d] * xv_re;
    const double b_im = k * ci + VN[2 * d + 1] - xh[d] * xv_im;
    // -(i/4pi)(b_re + i b_im) = (b_im - i b_re)/(4pi)
    out[2 * d] = b_im * INV_FOUR_PI;
    out[2 * d + 1] = -b_re * INV_FOUR_PI;
  }
}

__global__ void k_far_finish(const double* part, int nseg, double k, const double* obs, int nobs, int nrhs,
                             double* Fout) {
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (tid >= int64_t(nobs) * nrhs) return;
  const int o = int(tid % nobs), r = int(tid / nobs);
  const double xh[3] = {obs[3 * o], obs[3 * o + 1], obs[3 * o + 2]};
  double V[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int sg = 0; sg < nseg; ++sg) {
    const double* pp = part + (int64_t(r) * nseg + sg) * 12 * int64_t(nobs) + o;
    for (int c = 0; c < 12; ++c) V[c] += pp[int64_t(c) * nobs];
  }
  far_from_sums(xh, V, k, Fout + 6 * (int64_t(r) * nobs + o));
}

// Antipodal pairs: part[((r nseg + s) 24 + 4 comp + 2 trig + part) nh + o]
// holds the K split s of sum_p {cos, sin}(-k xh_o . y_p) {Re, Im} J_comp(y_p).
// With phase cos + i sin at xh and cos - i sin at -xh:
//   V(xh)  = (cc - ss) + i (cs + sc),   V(-xh) = (cc + ss) + i (cs - sc)
// (cc = cos Re J, cs = cos Im J, sc = sin Re J, ss = sin Im J).  Writes F at
// direction o and nh + o of the 2 nh per rhs.
__global__ void k_far_finish_pair(const double* part, int nseg, double k, const double* obs, int nh, int nrhs,
                                  double* Fout) {
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (tid >= int64_t(nh) * nrhs) return;
  const int o = int(tid % nh), r = int(tid / nh);
  double P[24];
  for (int c = 0; c < 24; ++c) P[c] = 0.0;
  for (int sg = 0; sg < nseg; ++sg) {
    const double* pp = part + (int64_t(r) * nseg + sg) * 24 * int64_t(nh) + o;
    for (int c = 0; c < 24; ++c) P[c] += pp[int64_t(c) * nh];
  }
  double Vp[12], Vm[12];
  for (int c = 0; c < 6; ++c) {
    const double cc = P[4 * c], cs = P[4 * c + 1], sc = P[4 * c + 2], ss = P[4 * c + 3];
    Vp[2 * c] = cc - ss;
    Vp[2 * c + 1] = cs + sc;
    Vm[2 * c] = cc + ss;
    Vm[2 * c + 1] = cs - sc;
  }
  const double xp[3] = {obs[3 * o], obs[3 * o + 1], obs[3 * o + 2]};
  const double xm[3] = {-xp[0], -xp[1], -xp[2]};
  double* out = Fout + 6 * (int64_t(r) * 2 * nh + o);
  far_from_sums(xp, Vp, k, out);
  far_from_sums(xm, Vm, k, out + 6 * int64_t(nh));
}

FarPlan far_field_plan(int F, int nrhs, int nobs) {
  FarPlan p;
  p.npts = int64_t(F) * 6;
  const int64_t oblocks = (nobs + FAR_BLOCK - 1) / FAR_BLOCK;
  // about 8 waves per SIMD over the chip, at least one LDS tile per segment
  const int64_t want = (8 * 1024 + oblocks * nrhs * (FAR_BLOCK / 64) - 1) / (oblocks * nrhs * (FAR_BLOCK / 64));
  const int64_t max_seg = (p.npts + FAR_TILE - 1) / FAR_TILE;
  p.nseg = int(std::max<int64_t>(1, std::min<int64_t>(want, max_seg)));
  p.seg_len = (p.npts + p.nseg - 1) / p.nseg;
  p.seg_len = (p.seg_len + FAR_TILE - 1) / FAR_TILE * FAR_TILE;
  p.nseg = int((p.npts + p.seg_len - 1) / p.seg_len);
  p.n_ypts = 4 * p.npts;
  p.n_J = 12 * p.npts * nrhs;
  p.n_part = int64_t(nrhs) * p.nseg * 12 * nobs;
  return p;
}

// The same plan with at most max_part partial-sum values: fewer, longer
// segments (whole LDS tiles) when the default split would exceed it.  The
// result may still exceed max_part with a single segment; callers check.
FarPlan far_field_plan_capped(int F, int nrhs, int nobs, int64_t max_part) {
  FarPlan p = far_field_plan(F, nrhs, nobs);
  if (p.n_part <= max_part) return p;
  const int64_t per_seg = int64_t(nrhs) * 12 * nobs;
  const int64_t nseg = std::max<int64_t>(1, max_part / per_seg);
  p.seg_len = (p.npts + nseg - 1) / nseg;
  p.seg_len = (p.seg_len + FAR_TILE - 1) / FAR_TILE * FAR_TILE;
  p.nseg = int((p.npts + p.seg_len - 1) / p.seg_len);
  p.n_part = per_seg * p.nseg;
  return p;
}

void launch_far_field(const AsmParams<double>& geo, const double* x, int64_t E_tot, int nrhs, double k,
                      const double* obs, int nobs, double* F_out, const FarPlan& plan, double* ypts, double* J,
                      double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_far_points, dim3(unsigned((plan.npts + 255) / 256)), dim3(256), 0, st, geo, x, E_tot, nrhs,
                     plan.npts, ypts, J);
  hipLaunchKernelGGL(k_far_sum, dim3(unsigned((nobs + FAR_BLOCK - 1) / FAR_BLOCK), unsigned(plan.nseg), unsigned(nrhs)),
                     dim3(FAR_BLOCK), 0, st, ypts, J, plan.npts, plan.seg_len, plan.nseg, k, obs, nobs, part);
  const int64_t n = int64_t(nobs) * nrhs;
  hipLaunchKernelGGL(k_far_finish, dim3(unsigned((n + 127) / 128)), dim3(128), 0, st, part, plan.nseg, k, obs, nobs,
                     nrhs, F_out);
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
