// Total electric field at points near and inside the scatterers (the
// Stratton-Chu representation of Section 2 with the solved traces):
//   outside:      E = E^inc - sum_m [ H^e(gamma_D E^s) + E^e(gamma_N E^s) ],  k = k_e,
//   inside m:     E = H^i_m(gamma_D E^i) + E^i_m(gamma_N E^i),                 k = k_m,
// with E v(x) = ik int v G - (1/ik) grad_x int div v G and
// H v(x) = int grad_x G x v, grad_x G = (x - y)(ik r - 1) G / r^2.  The traces
// are RT0 fields: the scaled unknowns u^s = [gamma_D E^s; k_e gamma_N E^s]
// outside, and u^s plus the L2 projection of u^inc onto RWG for the interior
// traces [gamma_D E^i; k_m gamma_N E^i].
//   pass 0: region of every point (solid angle of each closed surface:
//           4 pi inside, 0 outside; Van Oosterom and Strackee's formula);
//   pass 1: per point y of the 6-point rule on every triangle, the weighted
//           currents and surface divergences of both trace sets;
//   pass 2: per (point, right-hand side), the sums over the rule points
//           (tiles staged in LDS).
#include "common.hpp"
#include "kernels.hpp"

namespace pmchwt {

constexpr int NEAR_TILE = 128;
constexpr int NEAR_J = 28;  // doubles per (rhs, rule point): w J_D, w J_N, w div J_N for u^s, then for u^i

__global__ __launch_bounds__(256) void k_near_region(AsmParams<double> g, const int32_t* tri_off, int nscat,
                                                     const double* pts, int npts, int32_t* region) {
  __shared__ double tv[256][9];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const bool live = i < npts;
  double x[3] = {0, 0, 0};
  if (live)
    for (int d = 0; d < 3; ++d) x[d] = pts[3 * i + d];
  int reg = -1;
  const int F = g.F;
  for (int m = 0; m < nscat; ++m) {
    double tot = 0.0;
    for (int t0 = tri_off[m]; t0 < tri_off[m + 1]; t0 += 256) {
      const int nt = min(256, tri_off[m + 1] - t0);
      __syncthreads();
      if (threadIdx.x < nt)
        for (int q = 0; q < 9; ++q) tv[threadIdx.x][q] = g.tv[q * F + t0 + threadIdx.x];
      __syncthreads();
      for (int t = 0; t < nt; ++t) {
        double R[3][3];
        for (int k = 0; k < 3; ++k)
          for (int d = 0; d < 3; ++d) R[k][d] = tv[t][3 * k + d] - x[d];
        const double n1 = sqrt(R[0][0] * R[0][0] + R[0][1] * R[0][1] + R[0][2] * R[0][2]);
        const double n2 = sqrt(R[1][0] * R[1][0] + R[1][1] * R[1][1] + R[1][2] * R[1][2]);
        const double n3 = sqrt(R[2][0] * R[2][0] + R[2][1] * R[2][1] + R[2][2] * R[2][2]);
        const double cx = R[1][1] * R[2][2] - R[1][2] * R[2][1], cy = R[1][2] * R[2][0] - R[1][0] * R[2][2],
                     cz = R[1][0] * R[2][1] - R[1][1] * R[2][0];
        const double num = R[0][0] * cx + R[0][1] * cy + R[0][2] * cz;
        const double d12 = R[0][0] * R[1][0] + R[0][1] * R[1][1] + R[0][2] * R[1][2];
        const double d13 = R[0][0] * R[2][0] + R[0][1] * R[2][1] + R[0][2] * R[2][2];
        const double d23 = R[1][0] * R[2][0] + R[1][1] * R[2][1] + R[1][2] * R[2][2];
        tot += 2.0 * atan2(num, n1 * n2 * n3 + d12 * n3 + d13 * n2 + d23 * n1);
      }
    }
    if (fabs(tot) > 6.283185307179586) reg = m;
  }
  if (live) region[i] = reg;
}

// y and scatterer of every rule point; J[(r npts + q) NEAR_J + c]
__global__ void k_near_points(AsmParams<double> g, const double* x, const double* cinc, int64_t E_tot, int nrhs,
                              int64_t nq, double* ypts, double* J) {
  const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (tid >= nq) return;
  const int F = g.F;
  const int off = c_rule_off[4], nr = c_rule_n[4];
  const int T = int(tid / nr), q = int(tid % nr);
  double P[3][3];
  for (int k = 0; k < 3; ++k)
    for (int d = 0; d < 3; ++d) P[k][d] = g.tv[(3 * k + d) * F + T];
  const double A = g.tarea[T];
  double y[3];
  for (int d = 0; d < 3; ++d)
    y[d] = c_rule_l[off + q][0] * P[0][d] + c_rule_l[off + q][1] * P[1][d] + c_rule_l[off + q][2] * P[2][d];
  for (int d = 0; d < 3; ++d) ypts[4 * tid + d] = y[d];
  ypts[4 * tid + 3] = double(g.tscat[T]);
  const double wq = c_rule_w[off + q] * A;
  for (int r = 0; r < nrhs; ++r) {
    double v[NEAR_J];
    for (int c = 0; c < NEAR_J; ++c) v[c] = 0.0;
    for (int set = 0; set < 2; ++set) {
      const double* xD = x + 2 * (int64_t(r) * 2 * E_tot);
      const double* xN = xD + 2 * E_tot;
      const double* iD = cinc + 2 * (int64_t(r) * 2 * E_tot);
      const double* iN = iD + 2 * E_tot;
      double* o = v + 14 * set;
      for (int a = 0; a < 3; ++a) {
        const int e = g.t2e[a * F + T];
        const double s = g.tsgn[a * F + T];
        double dr = xD[2 * e], di = xD[2 * e + 1], nrr = xN[2 * e], ni = xN[2 * e + 1];
        if (set == 1) {
          dr += iD[2 * e];
          di += iD[2 * e + 1];
          nrr += iN[2 * e];
          ni += iN[2 * e + 1];
        }
        for (int d = 0; d < 3; ++d) {
          const double f = wq * s * (y[d] - P[a][d]) / (2.0 * A);
          o[2 * d] += f * dr;
          o[2 * d + 1] += f * di;
          o[6 + 2 * d] += f * nrr;
          o[6 + 2 * d + 1] += f * ni;
        }
        o[12] += wq * s / A * nrr;
        o[13] += wq * s / A * ni;
      }
    }
    double* out = J + NEAR_J * (int64_t(r) * nq + tid);
    for (int c = 0; c < NEAR_J; ++c) out[c] = v[c];
  }
}

// grid (point blocks of 256, rhs)
__global__ __launch_bounds__(256) void k_near_sum(const double* ypts, const double* J, int64_t nq, double k_ext,
                                                  const double* k_int, const double* pts, int npts,
                                                  const int32_t* region, const double* dirs, const double* pols,
                                                  double* Eout) {
  __shared__ double s_y[NEAR_TILE][4];
  __shared__ double s_j[NEAR_TILE][NEAR_J];
  const int i = blockIdx.x * 256 + threadIdx.x, r = blockIdx.y;
  const bool live = i < npts;
  double x[3] = {0, 0, 0};
  int reg = -1;
  if (live) {
    for (int d = 0; d < 3; ++d) x[d] = pts[3 * i + d];
    reg = region[i];
  }
  const double kr = reg < 0 ? k_ext : k_int[2 * reg], ki = reg < 0 ? 0.0 : k_int[2 * reg + 1];
  const bool decay = ki != 0.0;
  const int set = reg < 0 ? 0 : 1;
  // 1/k (complex) scales the Neumann-trace terms
  const double k2 = kr * kr + ki * ki, ikr = kr / k2, iki = -ki / k2;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const double* Jr = J + NEAR_J * (int64_t(r) * nq);
  for (int64_t t0 = 0; t0 < nq; t0 += NEAR_TILE) {
    const int nt = int(min<int64_t>(NEAR_TILE, nq - t0));
    __syncthreads();
    for (int q = threadIdx.x; q < nt * 4; q += 256) s_y[q >> 2][q & 3] = ypts[4 * t0 + q];
    for (int q = threadIdx.x; q < nt * NEAR_J; q += 256) s_j[q / NEAR_J][q % NEAR_J] = Jr[NEAR_J * t0 + q];
    __syncthreads();
    if (!live) continue;
    for (int t = 0; t < nt; ++t) {
      if (reg >= 0 && int(s_y[t][3]) != reg) continue;  // interior field: the own surface only
      const double dx = x[0] - s_y[t][0], dy = x[1] - s_y[t][1], dz = x[2] - s_y[t][2];
      const double r2 = dx * dx + dy * dy + dz * dz;
      const KernelVal<double> kv = helmholtz<double>(r2, kr, ki, decay, 1.0);  // G and (ikr - 1) G / r^2
      const double* v = s_j[t] + 14 * set;
      const double gd[3] = {dx, dy, dz};
      // H: grad G x J_D, grad G = Fg d
      for (int d = 0; d < 3; ++d) {
        const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
        // (d x J)_d = d_d1 J_d2 - d_d2 J_d1 (J complex)
        const double cr = gd[d1] * v[2 * d2] - gd[d2] * v[2 * d1];
        const double ci = gd[d1] * v[2 * d2 + 1] - gd[d2] * v[2 * d1 + 1];
        acc[2 * d] += kv.Fg.re * cr - kv.Fg.im * ci;
        acc[2 * d + 1] += kv.Fg.re * ci + kv.Fg.im * cr;
      }
      // E of J_N / k: ik G J_N / k - (1/(ik)) div(J_N)/k grad G = i G J_N - (1/(i k^2)) div grad G
      const double dvr = v[12], dvi = v[13];
      // c = div / k^2 ... (1/(ik)) (div/k) = -i div / k^2
      const double ik2r = ikr * ikr - iki * iki, ik2i = 2.0 * ikr * iki;  // 1/k^2
      const double er = dvr * ik2r - dvi * ik2i, ei = dvr * ik2i + dvi * ik2r;  // div / k^2
      // -(1/(i)) (div/k^2) = i (div/k^2): coefficient of grad G = Fg d
      const double gr = -ei, gi = er;  // i * (div/k^2)
      const double fgr = kv.Fg.re * gr - kv.Fg.im * gi, fgi = kv.Fg.re * gi + kv.Fg.im * gr;
      for (int d = 0; d < 3; ++d) {
        const double jr = v[6 + 2 * d], ji = v[6 + 2 * d + 1];
        // i G J_N
        acc[2 * d] += -(kv.G.re * ji + kv.G.im * jr);
        acc[2 * d + 1] += kv.G.re * jr - kv.G.im * ji;
        acc[2 * d] += fgr * gd[d];
        acc[2 * d + 1] += fgi * gd[d];
      }
    }
  }
  if (!live) return;
  double* o = Eout + 6 * (int64_t(r) * npts + i);
  if (reg >= 0) {
    for (int c = 0; c < 6; ++c) o[c] = acc[c];
    return;
  }
  // outside: E^inc - (H + E)
  const double ph = k_ext * (dirs[3 * r] * x[0] + dirs[3 * r + 1] * x[1] + dirs[3 * r + 2] * x[2]);
  double sn, cs;
  sincos_taylor(ph, &sn, &cs);
  for (int d = 0; d < 3; ++d) {
    const double pr = pols[6 * r + 2 * d], pi = pols[6 * r + 2 * d + 1];
    o[2 * d] = pr * cs - pi * sn - acc[2 * d];
    o[2 * d + 1] = pr * sn + pi * cs - acc[2 * d + 1];
  }
}

void launch_near_field(const AsmParams<double>& g, const int32_t* tri_off, int nscat, const double* x,
                       const double* cinc, int64_t E_tot, int nrhs, const double* pts, int npts,
                       const double* dirs, const double* pols, double k_ext, const double* k_int, int32_t* region,
                       double* ypts, double* J, double* Eout, hipStream_t st) {
  const int64_t nq = int64_t(g.F) * 6;
  hipLaunchKernelGGL(k_near_region, dim3(unsigned((npts + 255) / 256)), dim3(256), 0, st, g, tri_off, nscat, pts, npts,
                     region);
  hipLaunchKernelGGL(k_near_points, dim3(unsigned((nq + 255) / 256)), dim3(256), 0, st, g, x, cinc, E_tot, nrhs, nq,
                     ypts, J);
  hipLaunchKernelGGL(k_near_sum, dim3(unsigned((npts + 255) / 256), unsigned(nrhs)), dim3(256), 0, st, ypts, J, nq,
                     k_ext, k_int, pts, npts, region, dirs, pols, Eout);
}

int near_j_doubles() { return NEAR_J; }

}  // namespace pmchwt
