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
// The Galerkin blocks of S and C are symmetric (swapping the test and the
// trial function swaps the two integration variables; for C both the
// gradient and the triple product change sign), and the regular pairs' rule
// is the same tensor rule in either order.  So every unordered regular pair
// is integrated once and used both ways:
//   pass 1 (k_free_tiles): upper tiles (I, J) of 64 x 64 triangles; wave w
//   takes test triangles 16 w .. 16 w + 15 of tile I one at a time against
//   the 64 trial triangles of tile J (one per lane; on diagonal tiles only
//   the pairs above the diagonal).  For each pair and wavenumber the kernel
//   moments give the 3 x 3 blocks S_ab, C_ab, which add
//     yD[a] += C xD[b] + S/k xN[b],   yN[a] += C xN[b] - k S xD[b]
//   to the test triangle's bases a (summed over the wave) and the same with
//   a and b exchanged to the trial triangle's bases b (summed per lane over
//   the wave's test triangles, then over the four wavefronts in order).
//   The sums of tile I's triangles from tile J land at part[I][J], those of
//   tile J's triangles at part[J][I] (diagonal tiles: row plus column sums).
//   pass 2 (k_free_sing_sum): per triangle, its vertex-sharing pairs from
//   the singular kernel's FP64 blocks, plus the partial sums part[K][0..nt)
//   in order, into one (yD, yN) per slot (rhs, t, a).
//   pass 3 (k_free_combine): the two slots of every edge (T+ and T- carry
//   the RWG signs already).
// Exterior operators (k_e) act on every pair, interior ones (k_m) on pairs
// of one scatterer.
#include "common.hpp"
#include "kernels.hpp"

namespace pmchwt {

constexpr int FREE_TT = 64;                       // triangles per tile side
constexpr int FREE_WAVES = 4;                     // wavefronts per workgroup
constexpr int FREE_STEPS = FREE_TT / FREE_WAVES;  // test triangles per wavefront

// sum over the 64 lanes (DPP within rows of 16, then across rows); every
// lane gets it, in the same order on every lane
__device__ __forceinline__ double wave_sum_free(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  v += dpp_move<0x140>(v);  // row_mirror
  v += __shfl_xor(v, 16, WAVE);
  v += __shfl_xor(v, 32, WAVE);
  return v;
}

// row-major index t of the upper tiles (I <= J) of an nt x nt grid -> (I, J);
// row I starts at I nt - I (I - 1) / 2
__device__ __forceinline__ void upper_tile(int t, int nt, int& I, int& J) {
  const double b = 2.0 * nt + 1.0;
  int i = int((b - sqrt(b * b - 8.0 * double(t))) * 0.5);
  i = max(0, min(i, nt - 1));
  while (i > 0 && i * nt - i * (i - 1) / 2 > t) --i;
  while (i + 1 < nt && (i + 1) * nt - (i + 1) * i / 2 <= t) ++i;
  I = i;
  J = i + (t - (i * nt - i * (i - 1) / 2));
}

// (yD, yN) of one basis += C (xD, xN) + S (g1 xN, g2 xD) into o[0..3]
__device__ __forceinline__ void free_add(double* o, const cplx<double>& S, const cplx<double>& C,
                                         const cplx<double>& g1, const cplx<double>& g2, const cplx<double>& xD,
                                         const cplx<double>& xN) {
  const cplx<double> a1 = cmul(C, xD), a2 = cmul(S, cmul(g1, xN));
  const cplx<double> b1 = cmul(C, xN), b2 = cmul(S, cmul(g2, xD));
  o[0] += a1.re + a2.re;
  o[1] += a1.im + a2.im;
  o[2] += b1.re + b2.re;
  o[3] += b1.im + b2.im;
}

// grid (upper tiles, nrhs); part: [rhs][K][L][64][12] (12 = 3 bases x yD, yN complex)
__global__ __launch_bounds__(FREE_WAVES * WAVE, 2) void k_free_tiles(AsmParams<double> p, FreeJob f, int nt,
                                                                     double* __restrict__ part) {
  __shared__ double s_x[FREE_TT][14][4];              // test rule points (relative to the centroid), weight x area
  __shared__ double s_a[FREE_TT][3][4];               // test bases: alpha, alpha (v_a - c1)
  __shared__ double s_c[FREE_TT][4];                  // centroid, diameter^2
  __shared__ int s_v[FREE_TT][4];                     // vertex ids, scatterer
  __shared__ double s_row[FREE_TT][12];               // test triangles' sums
  __shared__ double s_col[FREE_WAVES][FREE_TT][12];   // trial triangles' sums per wavefront
  __shared__ double s_tv2[FREE_TT][3][4];             // trial triangles: vertices, alpha of each basis
  __shared__ int s_e2[FREE_TT][3];                    // trial triangles' basis edges
  __shared__ double s_x1[FREE_WAVES][3][8];           // per wavefront, its test triangle's bases: xD, xN, uD, uN
  int I, J;
  upper_tile(blockIdx.x, nt, I, J);
  const int r = blockIdx.y;
  const int F = p.F, E = f.E_tot;
  const double* xr = f.x + 2 * int64_t(r) * f.vs;
  const double* ur = (f.xi ? f.xi : f.x) + 2 * int64_t(r) * f.vs;
  // test tile data
  for (int i = threadIdx.x; i < FREE_TT * 14; i += blockDim.x) {
    const int lt = i / 14, q = i % 14, t1 = min(I * FREE_TT + lt, F - 1);
    double c[3];
    for (int d = 0; d < 3; ++d) c[d] = p.tcen[d * F + t1];
    for (int d = 0; d < 3; ++d) {
      double x = 0.0;
      for (int k = 0; k < 3; ++k) x += c_rule_l[q][k] * (p.tv[(3 * k + d) * F + t1] - c[d]);
      s_x[lt][q][d] = x;
    }
    s_x[lt][q][3] = c_rule_w[q] * p.tarea[t1];
  }
  for (int i = threadIdx.x; i < FREE_TT * 3; i += blockDim.x) {
    const int lt = i / 3, a = i % 3, t1 = min(I * FREE_TT + lt, F - 1);
    const double al = p.tsgn[a * F + t1] / (2.0 * p.tarea[t1]);
    s_a[lt][a][0] = al;
    for (int d = 0; d < 3; ++d) s_a[lt][a][1 + d] = al * (p.tv[(3 * a + d) * F + t1] - p.tcen[d * F + t1]);
  }
  for (int i = threadIdx.x; i < FREE_WAVES * FREE_TT * 12; i += blockDim.x) (&s_col[0][0][0])[i] = 0.0;
  for (int i = threadIdx.x; i < FREE_TT * 3; i += blockDim.x) {
    const int lt = i / 3, b = i % 3, t2 = min(J * FREE_TT + lt, F - 1);
    for (int d = 0; d < 3; ++d) s_tv2[lt][b][d] = p.tv[(3 * b + d) * F + t2];
    s_tv2[lt][b][3] = p.tsgn[b * F + t2] / (2.0 * p.tarea[t2]);
    s_e2[lt][b] = p.t2e[b * F + t2];
  }
  for (int lt = threadIdx.x; lt < FREE_TT; lt += blockDim.x) {
    const int t1 = min(I * FREE_TT + lt, F - 1);
    for (int d = 0; d < 3; ++d) s_c[lt][d] = p.tcen[d * F + t1];
    s_c[lt][3] = p.tdiam2[t1];
    for (int k = 0; k < 3; ++k) s_v[lt][k] = p.tvid[k * F + t1];
    s_v[lt][3] = p.tscat[t1];
  }
  __syncthreads();

  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  const int t2 = J * FREE_TT + lane;
  const bool v2 = t2 < F;
  const int t2c = v2 ? t2 : F - 1;
  const double c2[3] = {p.tcen[t2c], p.tcen[F + t2c], p.tcen[2 * F + t2c]};
  const double A2 = p.tarea[t2c], d2 = p.tdiam2[t2c];
  const int vb0 = p.tvid[t2c], vb1 = p.tvid[F + t2c], vb2 = p.tvid[2 * F + t2c], s2 = p.tscat[t2c];
  const double ke = p.k_ext;
  double* col = s_col[w][lane];  // this lane's trial triangle, summed over the wave's test triangles

  for (int st = 0; st < FREE_STEPS; ++st) {
    const int lt1 = w * FREE_STEPS + st, t1 = I * FREE_TT + lt1;
    double row[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) row[q] = 0.0;
    // the exterior and interior inputs at the test triangle's three edges,
    // once per step into this wavefront's slot (lane 8 a + c: basis a,
    // c = xD re, im, xN re, im, uD re, im, uN re, im)
    if (lane < 24) {
      const int a = lane >> 3, c = lane & 7, e = p.t2e[a * F + min(t1, F - 1)];
      const double* src = c < 4 ? xr : ur;
      s_x1[w][a][c] = src[2 * ((c & 2) ? E + e : e) + (c & 1)];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    bool live = v2 && t1 < F && (I != J || lane > lt1);
    if (live) {
      const int va0 = s_v[lt1][0], va1 = s_v[lt1][1], va2 = s_v[lt1][2];
      const bool shared = vb0 == va0 || vb0 == va1 || vb0 == va2 || vb1 == va0 || vb1 == va1 || vb1 == va2 ||
                          vb2 == va0 || vb2 == va1 || vb2 == va2;
      live = !shared;  // vertex-sharing pairs: the singular kernel's FP64 blocks, in pass 2
    }
    if (live) {
      const double c1[3] = {s_c[lt1][0], s_c[lt1][1], s_c[lt1][2]};
      const int s1 = s_v[lt1][3];
      const int cls = classify_pair(c1[0], c1[1], c1[2], c2[0], c2[1], c2[2], s_c[lt1][3], d2);
      const int qr = cls == 0 ? p.q_near : (cls == 1 ? p.q_medium : p.q_far);
      const int off = c_rule_off[qr], n = c_rule_n[qr];
      double P2[3][3];
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int d = 0; d < 3; ++d) P2[k][d] = s_tv2[lane][k][d] - c1[d];
      for (int kk = f.use_ext ? 0 : 1; kk < 2; ++kk) {
        if (kk == 1 && s2 != s1) break;  // interior operators: one scatterer
        const double kr = kk == 0 ? ke : p.k_int[2 * s1], ki = kk == 0 ? 0.0 : p.k_int[2 * s1 + 1];
        const bool decay = kk == 1 && ki != 0.0;
        const double ik2 = 1.0 / (kr * kr + ki * ki);
        // combination factors 1/k and -k
        const cplx<double> g1 = {kr * ik2, -ki * ik2}, g2 = {-kr, -ki};
        const double* xin = kk == 0 ? xr : ur;
        Moments<double> mm;
        mm.zero();
#pragma unroll 1
        for (int a = 0; a < n; ++a) {
          const double x[3] = {s_x[lt1][off + a][0], s_x[lt1][off + a][1], s_x[lt1][off + a][2]};
          const double wa = s_x[lt1][off + a][3] * A2;
#pragma unroll 1
          for (int b = 0; b < n; ++b) {
            double y[3];
            const double lb0 = c_rule_l[off + b][0], lb1 = c_rule_l[off + b][1], lb2 = c_rule_l[off + b][2];
#pragma unroll
            for (int d = 0; d < 3; ++d) y[d] = lb0 * P2[0][d] + lb1 * P2[1][d] + lb2 * P2[2][d];
            const double wgt = wa * c_rule_w[off + b];
            const double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
            mm.add(helmholtz<double>(dx * dx + dy * dy + dz * dz, kr, ki, decay, wgt), x, y, true);
          }
        }
        // contraction against the RT0 fields of both triangles, one trial basis
        // b at a time:
        //   Sv = a1 a2 Mxy - a1 (w2.Mx) - a2 (w1.My) + (w1.w2) M0,  Sd = 4 a1 a2 M0,
        //   S = -ik Sv - Sd/(ik),  C = -[a1 (w2.Nx) - a2 (w1.Nx) + w1.(Nd x w2)]
#pragma unroll 1
        for (int b = 0; b < 3; ++b) {
          const int jb = s_e2[lane][b];
          const double al2 = s_tv2[lane][b][3];
          double w2[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) w2[d] = al2 * (s_tv2[lane][b][d] - c1[d]);
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
          const cplx<double> xbD = {xin[2 * jb], xin[2 * jb + 1]};
          const cplx<double> xbN = {xin[2 * (E + jb)], xin[2 * (E + jb) + 1]};
          double cb[4] = {0.0, 0.0, 0.0, 0.0};  // trial basis b's sum over the test bases
#pragma unroll 1
          for (int a = 0; a < 3; ++a) {
            const double al1 = s_a[lt1][a][0];
            const double w1[3] = {s_a[lt1][a][1], s_a[lt1][a][2], s_a[lt1][a][3]};
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
            double ra[4] = {0.0, 0.0, 0.0, 0.0};
            free_add(ra, S, C, g1, g2, xbD, xbN);
            // static register indices (a is a loop counter)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              row[q] += a == 0 ? ra[q] : 0.0;
              row[4 + q] += a == 1 ? ra[q] : 0.0;
              row[8 + q] += a == 2 ? ra[q] : 0.0;
            }
            const double* xa = s_x1[w][a] + 4 * kk;
            free_add(cb, S, C, g1, g2, cplx<double>{xa[0], xa[1]}, cplx<double>{xa[2], xa[3]});
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) col[4 * b + q] += cb[q];
        }
      }
    }
    // the test triangle's sums over the wave's 64 trial triangles
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      const double v = wave_sum_free(row[q]);
      if (lane == 0) s_row[lt1][q] = v;
    }
  }
  __syncthreads();
  double* pr = part + int64_t(r) * nt * nt * FREE_TT * 12;
  {
    double* o = pr + (int64_t(J) * nt + I) * FREE_TT * 12;
    for (int i = threadIdx.x; i < FREE_TT * 12; i += blockDim.x) {
      const int l = i / 12, q = i % 12;
      double v = s_col[0][l][q];
#pragma unroll
      for (int u = 1; u < FREE_WAVES; ++u) v += s_col[u][l][q];
      if (I == J) v = s_row[l][q] + v;
      o[i] = v;
    }
  }
  if (I != J) {
    double* o = pr + (int64_t(I) * nt + J) * FREE_TT * 12;
    for (int i = threadIdx.x; i < FREE_TT * 12; i += blockDim.x) o[i] = s_row[i / 12][i % 12];
  }
}

// grid (F, nrhs), one wavefront: the vertex-sharing pairs of test triangle
// t1 (lanes over its pairs; the FP64 blocks of the singular kernel), summed
// over the wave, then the regular pairs' partial sums of its tile row in
// order; one (yD, yN) per slot (rhs, t1, a).
__global__ __launch_bounds__(WAVE) void k_free_sing_sum(AsmParams<double> p, FreeJob f, int nt,
                                                        const double* __restrict__ part) {
  const int t1 = blockIdx.x, r = blockIdx.y, lane = threadIdx.x;
  const int F = p.F, E = f.E_tot;
  const int s1 = p.tscat[t1];
  const double ke = p.k_ext;
  const double kir = p.k_int[2 * s1], kii = p.k_int[2 * s1 + 1];
  const double kim2 = kir * kir + kii * kii;
  const cplx<double> fe1 = {1.0 / ke, 0.0}, fe2 = {-ke, 0.0};
  const cplx<double> fi1 = {kir / kim2, -kii / kim2}, fi2 = {-kir, -kii};
  const double* xr = f.x + 2 * int64_t(r) * f.vs;
  const double* ur = (f.xi ? f.xi : f.x) + 2 * int64_t(r) * f.vs;
  double acc[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) acc[q] = 0.0;
  const int64_t sp0 = f.sing_ptr[t1], sp1 = f.sing_ptr[t1 + 1];
  for (int64_t sp = sp0 + lane; sp < sp1; sp += WAVE) {
    const int t2 = f.sing_pairs[2 * sp + 1];
    const cplx<double>* blk = reinterpret_cast<const cplx<double>*>(f.sing_blk) + sp * 36;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const int e = p.t2e[b * F + t2];
      const cplx<double> xD = {xr[2 * e], xr[2 * e + 1]}, xN = {xr[2 * (E + e)], xr[2 * (E + e) + 1]};
      const cplx<double> uD = {ur[2 * e], ur[2 * e + 1]}, uN = {ur[2 * (E + e)], ur[2 * (E + e) + 1]};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const cplx<double>* en = blk + 4 * (3 * a + b);
        if (f.use_ext) free_add(acc + 4 * a, en[0], en[1], fe1, fe2, xD, xN);
        free_add(acc + 4 * a, en[2], en[3], fi1, fi2, uD, uN);
      }
    }
  }
  double tot[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) tot[q] = wave_sum_free(acc[q]);
  if (lane < 12) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < 12; ++q) v = q == lane ? tot[q] : v;
    const int K = t1 / FREE_TT, tl = t1 - K * FREE_TT;
    const double* pp = part + ((int64_t(r) * nt + K) * nt * FREE_TT + tl) * 12 + lane;
    for (int L = 0; L < nt; ++L) v += pp[int64_t(L) * FREE_TT * 12];
    // slot layout: [rhs][3F slots][yD re, yD im, yN re, yN im]
    f.slots[(int64_t(r) * 3 * F + 3 * int64_t(t1)) * 4 + lane] = v;
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

int free_tiles(int F) { return (F + FREE_TT - 1) / FREE_TT; }

int64_t free_part_doubles(int F, int nrhs) {
  const int64_t nt = free_tiles(F);
  return int64_t(nrhs) * nt * nt * FREE_TT * 12;
}

void launch_free_apply(const AsmParams<double>& p, const FreeJob& f, double* part, hipStream_t st) {
  const int nt = free_tiles(p.F);
  const int64_t nup = int64_t(nt) * (nt + 1) / 2;
  hipLaunchKernelGGL(k_free_tiles, dim3(unsigned(nup), unsigned(f.nrhs)), dim3(FREE_WAVES * WAVE), 0, st, p, f, nt,
                     part);
  hipLaunchKernelGGL(k_free_sing_sum, dim3(unsigned(p.F), unsigned(f.nrhs)), dim3(WAVE), 0, st, p, f, nt, part);
  const int64_t n = int64_t(f.E_tot) * f.nrhs;
  hipLaunchKernelGGL(k_free_combine, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, f, p.F);
}

}  // namespace pmchwt
