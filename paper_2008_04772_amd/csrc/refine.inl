// Matrix-free FP64 products with the PMCHWT operator (Section 2) for the
// iterative-refinement residual of a solve whose stored operators are FP32:
// r = b - A x with b = g/2 - A^i c_inc (Section 3.2) is g/2 - (A^i u + A^e x)
// with u = c_inc + x, one product whose exterior and interior operators read
// different inputs (x and xi).  Every entry is integrated again in FP64 with the same
// rules as the FP64 assembly (regular pairs: tensor symmetric rules by
// relative distance; singular pairs: the Sauter-Schwab values the singular
// kernel keeps in FP64), and contracted with x on the fly, so the product is
// that of the FP64 Galerkin matrix without storing it.
//
// Pass 1: one workgroup per test triangle t1 (and chunk of RC right-hand
// sides).  Its threads stride over the trial triangles; for each disjoint
// pair and each wavenumber they accumulate the kernel moments, contract them
// against the three RWG functions of either triangle and add
//   yD[a] += C xD[b] + S/k xN[b],   yN[a] += C xN[b] - k S xD[b]
// for every local test basis a of t1 (exterior k_e on every pair, interior
// k_m on pairs of one scatterer).  Pairs that share a vertex read their
// local blocks from the singular kernel's FP64 output.  The workgroup sums
// its threads' values in a fixed order and writes one (yD, yN) per slot
// (rhs, t1, a).  Pass 2 adds the two slots of every edge (T+ and T- carry the
// RWG signs already).
#include "common.hpp"
#include "kernels.hpp"

namespace pmchwt {

constexpr int FREE_THREADS = 256;

__device__ __forceinline__ double wave_sum_free(double v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// acc[r][a][0] = yD, acc[r][a][1] = yN (complex) += C x + S factors
template <int RC>
__device__ __forceinline__ void apply_block(cplx<double> (&acc)[RC][3][2], int a, const cplx<double>& S,
                                            const cplx<double>& C, const cplx<double>& f1, const cplx<double>& f2,
                                            const cplx<double> (&xD)[RC], const cplx<double> (&xN)[RC]) {
  const cplx<double> s1 = cmul(S, f1), s2 = cmul(S, f2);
#pragma unroll
  for (int r = 0; r < RC; ++r) {
    const cplx<double> a1 = cmul(C, xD[r]), a2 = cmul(s1, xN[r]);
    const cplx<double> b1 = cmul(C, xN[r]), b2 = cmul(s2, xD[r]);
    acc[r][a][0].re += a1.re + a2.re;
    acc[r][a][0].im += a1.im + a2.im;
    acc[r][a][1].re += b1.re + b2.re;
    acc[r][a][1].im += b1.im + b2.im;
  }
}

template <int RC>
__global__ __launch_bounds__(FREE_THREADS, 2) void k_free_apply(AsmParams<double> p, FreeJob f) {
  __shared__ double red[FREE_THREADS / WAVE][RC * 12];
  __shared__ double s_t1[3][4];  // per test basis a of t1: alpha, w (RT0 field alpha x - w)
  __shared__ double s_x[14][4];  // points of every triangle rule on t1 (relative to its centroid), weight x A1
  const int t1 = blockIdx.x;
  const int r0 = blockIdx.y * RC;
  const int F = p.F;
  const int s1 = p.tscat[t1];
  double c1[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) c1[d] = p.tcen[d * F + t1];
  int va[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) va[k] = p.tvid[k * F + t1];
  const double A1 = p.tarea[t1], d1 = p.tdiam2[t1];
  if (threadIdx.x < 3) {
    const int a = threadIdx.x;
    const double al = p.tsgn[a * F + t1] / (2.0 * A1);
    s_t1[a][0] = al;
    for (int d = 0; d < 3; ++d) s_t1[a][1 + d] = al * (p.tv[(3 * a + d) * F + t1] - c1[d]);
  } else if (threadIdx.x >= 32 && threadIdx.x < 46) {
    const int i = threadIdx.x - 32;
    for (int d = 0; d < 3; ++d) {
      double x = 0.0;
      for (int k = 0; k < 3; ++k) x += c_rule_l[i][k] * (p.tv[(3 * k + d) * F + t1] - c1[d]);
      s_x[i][d] = x;
    }
    s_x[i][3] = c_rule_w[i] * A1;
  }
  __syncthreads();
  const double ke = p.k_ext;
  const double kir = p.k_int[2 * s1], kii = p.k_int[2 * s1 + 1];
  // combination factors: 1/k and -k for the exterior and interior wavenumbers
  const cplx<double> fe1 = {1.0 / ke, 0.0}, fe2 = {-ke, 0.0};
  const double kim2 = kir * kir + kii * kii;
  const cplx<double> fi1 = {kir / kim2, -kii / kim2}, fi2 = {-kir, -kii};

  cplx<double> acc[RC][3][2];
#pragma unroll
  for (int r = 0; r < RC; ++r)
#pragma unroll
    for (int a = 0; a < 3; ++a) acc[r][a][0] = acc[r][a][1] = {0.0, 0.0};
  const int nr = min(RC, f.nrhs - r0);

  // one wavenumber per sweep over the trial triangles: only one set of
  // moments and the accumulators stay live
  for (int kk = f.use_ext ? 0 : 1; kk < 2; ++kk) {
    const double kr = kk == 0 ? ke : kir, ki = kk == 0 ? 0.0 : kii;
    const bool decay = kk == 1 && kii != 0.0;
    const double ik2 = 1.0 / (kr * kr + ki * ki);
    const cplx<double> g1 = kk == 0 ? fe1 : fi1, g2 = kk == 0 ? fe2 : fi2;
    const double* xin = (kk == 1 && f.xi) ? f.xi : f.x;
    for (int t2 = threadIdx.x; t2 < F; t2 += FREE_THREADS) {
      if (kk == 1 && p.tscat[t2] != s1) continue;  // interior operators: one scatterer
      bool shared = false;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int vb = p.tvid[k * F + t2];
        shared |= (vb == va[0]) | (vb == va[1]) | (vb == va[2]);
      }
      if (shared) continue;  // singular pair: read below from the FP64 blocks
      const int cls = classify_pair(c1[0], c1[1], c1[2], p.tcen[t2], p.tcen[F + t2], p.tcen[2 * F + t2], d1,
                                    p.tdiam2[t2]);
      const int q = cls == 0 ? p.q_near : (cls == 1 ? p.q_medium : p.q_far);
      const int off = c_rule_off[q], n = c_rule_n[q];
      double P2[3][3];
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int d = 0; d < 3; ++d) P2[k][d] = p.tv[(3 * k + d) * F + t2] - c1[d];
      const double A2 = p.tarea[t2];
      Moments<double> mm;
      mm.zero();
#pragma unroll 1
      for (int a = 0; a < n; ++a) {
        const double x[3] = {s_x[off + a][0], s_x[off + a][1], s_x[off + a][2]};
        const double wa = s_x[off + a][3] * A2;
#pragma unroll 1
        for (int b = 0; b < n; ++b) {
          double y[3];
          const double lb0 = c_rule_l[off + b][0], lb1 = c_rule_l[off + b][1], lb2 = c_rule_l[off + b][2];
#pragma unroll
          for (int d = 0; d < 3; ++d) y[d] = lb0 * P2[0][d] + lb1 * P2[1][d] + lb2 * P2[2][d];
          const double w = wa * c_rule_w[off + b];
          const double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
          const double r2 = dx * dx + dy * dy + dz * dz;
          mm.add(helmholtz<double>(r2, kr, ki, decay, w), x, y, true);
        }
      }
      // contraction against the RT0 fields of both triangles, one trial basis
      // b at a time (its b-only terms once, then the three test bases):
      //   Sv = a1 a2 Mxy - a1 (w2.Mx) - a2 (w1.My) + (w1.w2) M0,  Sd = 4 a1 a2 M0,
      //   S = -ik Sv - Sd/(ik),  C = -[a1 (w2.Nx) - a2 (w1.Nx) + w1.(Nd x w2)]
#pragma unroll 1
      for (int b = 0; b < 3; ++b) {
        const int jb = p.t2e[b * F + t2];
        const double al2 = p.tsgn[b * F + t2] / (2.0 * A2);
        double w2[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) w2[d] = al2 * (p.tv[(3 * b + d) * F + t2] - c1[d]);
        cplx<double> Pb = {0, 0}, Qb = {0, 0}, Rb[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          Pb.re += w2[d] * mm.Mx[d].re;
          Pb.im += w2[d] * mm.Mx[d].im;
          Qb.re += w2[d] * mm.Nx[d].re;
          Qb.im += w2[d] * mm.Nx[d].im;
        }
        Rb[0] = {mm.Nd[1].re * w2[2] - mm.Nd[2].re * w2[1], mm.Nd[1].im * w2[2] - mm.Nd[2].im * w2[1]};
        Rb[1] = {mm.Nd[2].re * w2[0] - mm.Nd[0].re * w2[2], mm.Nd[2].im * w2[0] - mm.Nd[0].im * w2[2]};
        Rb[2] = {mm.Nd[0].re * w2[1] - mm.Nd[1].re * w2[0], mm.Nd[0].im * w2[1] - mm.Nd[1].im * w2[0]};
        cplx<double> gxN[RC], gxD[RC], xD[RC], xN[RC];
#pragma unroll
        for (int r = 0; r < RC; ++r) {
          const double* xr = xin + 2 * (int64_t(r0 + (r < nr ? r : 0)) * f.vs);
          xD[r] = {xr[2 * jb], xr[2 * jb + 1]};
          xN[r] = {xr[2 * (f.E_tot + jb)], xr[2 * (f.E_tot + jb) + 1]};
          gxN[r] = cmul(g1, xN[r]);
          gxD[r] = cmul(g2, xD[r]);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const double al1 = s_t1[a][0];
          const double w1[3] = {s_t1[a][1], s_t1[a][2], s_t1[a][3]};
          cplx<double> Ua = {0, 0}, Va = {0, 0}, wR = {0, 0};
          double ww = 0.0;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            Ua.re += w1[d] * mm.My[d].re;
            Ua.im += w1[d] * mm.My[d].im;
            Va.re += w1[d] * mm.Nx[d].re;
            Va.im += w1[d] * mm.Nx[d].im;
            wR.re += w1[d] * Rb[d].re;
            wR.im += w1[d] * Rb[d].im;
            ww += w1[d] * w2[d];
          }
          const double aa = al1 * al2;
          const double sv_re = aa * mm.Mxy.re - al1 * Pb.re - al2 * Ua.re + ww * mm.M0.re;
          const double sv_im = aa * mm.Mxy.im - al1 * Pb.im - al2 * Ua.im + ww * mm.M0.im;
          const double sd_re = 4.0 * aa * mm.M0.re, sd_im = 4.0 * aa * mm.M0.im;
          const double t_re = (sd_re * kr + sd_im * ki) * ik2, t_im = (sd_im * kr - sd_re * ki) * ik2;
          const cplx<double> S = {ki * sv_re + kr * sv_im - t_im, ki * sv_im - kr * sv_re + t_re};
          const cplx<double> C = {-(al1 * Qb.re - al2 * Va.re + wR.re), -(al1 * Qb.im - al2 * Va.im + wR.im)};
#pragma unroll
          for (int r = 0; r < RC; ++r) {
            const cplx<double> a1 = cmul(C, xD[r]), a2 = cmul(S, gxN[r]);
            const cplx<double> b1 = cmul(C, xN[r]), b2 = cmul(S, gxD[r]);
            acc[r][a][0].re += a1.re + a2.re;
            acc[r][a][0].im += a1.im + a2.im;
            acc[r][a][1].re += b1.re + b2.re;
            acc[r][a][1].im += b1.im + b2.im;
          }
        }
      }
    }
  }

  // singular pairs of t1 (vertex-sharing, edge-sharing, identical)
  const int64_t sp0 = f.sing_ptr[t1], sp1 = f.sing_ptr[t1 + 1];
  for (int64_t sp = sp0 + threadIdx.x; sp < sp1; sp += FREE_THREADS) {
    const int t2 = f.sing_pairs[2 * sp + 1];
    int jb[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) jb[b] = p.t2e[b * F + t2];
    const cplx<double>* blk = reinterpret_cast<const cplx<double>*>(f.sing_blk) + sp * 36;
    const double* xin = f.xi ? f.xi : f.x;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      cplx<double> xD[RC], xN[RC], uD[RC], uN[RC];
#pragma unroll
      for (int r = 0; r < RC; ++r) {
        const int64_t ro = 2 * (int64_t(r0 + (r < nr ? r : 0)) * f.vs);
        const double* xr = f.x + ro;
        const double* ur = xin + ro;
        xD[r] = {xr[2 * jb[b]], xr[2 * jb[b] + 1]};
        xN[r] = {xr[2 * (f.E_tot + jb[b])], xr[2 * (f.E_tot + jb[b]) + 1]};
        uD[r] = {ur[2 * jb[b]], ur[2 * jb[b] + 1]};
        uN[r] = {ur[2 * (f.E_tot + jb[b])], ur[2 * (f.E_tot + jb[b]) + 1]};
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const cplx<double>* e = blk + 4 * (3 * a + b);
        if (f.use_ext) apply_block<RC>(acc, a, e[0], e[1], fe1, fe2, xD, xN);
        apply_block<RC>(acc, a, e[2], e[3], fi1, fi2, uD, uN);
      }
    }
  }

  // fixed-order reduction: lanes by butterfly, waves through LDS
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
#pragma unroll
  for (int r = 0; r < RC; ++r)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const double vr = wave_sum_free(acc[r][a][c].re), vi = wave_sum_free(acc[r][a][c].im);
        if (lane == 0) {
          red[wv][((r * 3 + a) * 2 + c) * 2] = vr;
          red[wv][((r * 3 + a) * 2 + c) * 2 + 1] = vi;
        }
      }
  __syncthreads();
  if (threadIdx.x < RC * 12) {
    const int r = threadIdx.x / 12, rest = threadIdx.x % 12;
    if (r < nr) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < FREE_THREADS / WAVE; ++w) s += red[w][threadIdx.x];
      // slot layout: [rhs][3F slots][yD re, yD im, yN re, yN im]
      const int a = rest / 4, c = rest % 4;
      f.slots[(int64_t(r0 + r) * 3 * F + 3 * int64_t(t1) + a) * 4 + c] = s;
    }
  }
}

// y[r][comp][i] = slot(T+(i)) + slot(T-(i)) for every union edge i
__global__ void k_free_combine(FreeJob f, int F) {
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (tid >= int64_t(f.E_tot) * f.nrhs) return;
  const int i = int(tid % f.E_tot), r = int(tid / f.E_tot);
  const int sp = f.edge_slots[2 * i], sm = f.edge_slots[2 * i + 1];
  const double* a = f.slots + (int64_t(r) * 3 * F + sp) * 4;
  const double* b = f.slots + (int64_t(r) * 3 * F + sm) * 4;
  double* y = f.y + 2 * (int64_t(r) * f.vs);
  y[2 * i] = a[0] + b[0];
  y[2 * i + 1] = a[1] + b[1];
  y[2 * (f.E_tot + i)] = a[2] + b[2];
  y[2 * (f.E_tot + i) + 1] = a[3] + b[3];
}

void launch_free_apply(const AsmParams<double>& p, const FreeJob& f, hipStream_t st) {
  // one right-hand side per workgroup: the variants with 2 or 4 exceed the
  // register file and spill (the integrals are the cost; callers with many
  // right-hand sides use an assembled FP64 operator instead)
  const int rc = 1;
  const dim3 grid{unsigned(p.F), unsigned((f.nrhs + rc - 1) / rc)};
  if (rc == 4)
    hipLaunchKernelGGL(k_free_apply<4>, grid, dim3(FREE_THREADS), 0, st, p, f);
  else if (rc == 2)
    hipLaunchKernelGGL(k_free_apply<2>, grid, dim3(FREE_THREADS), 0, st, p, f);
  else
    hipLaunchKernelGGL(k_free_apply<1>, grid, dim3(FREE_THREADS), 0, st, p, f);
  const int64_t n = int64_t(f.E_tot) * f.nrhs;
  hipLaunchKernelGGL(k_free_combine, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, f, p.F);
}

}  // namespace pmchwt
