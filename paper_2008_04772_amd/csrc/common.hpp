// Shared device helpers for the PMCHWT kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pmchwt {

constexpr int WAVE = 64;
constexpr double INV_FOUR_PI = 0.079577471545947667884441881686257;

template <typename R>
struct cplx {
  R re, im;
};

template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// Helmholtz kernel pieces at distance r for wavenumber k = kr + i ki:
//   G = w exp(ikr) / (4 pi r),  Fg = G (ikr - 1) / r^2, so grad_x G = Fg (x - y).
// `decay` selects the exp(-ki r) factor (ki == 0 for real exterior media).
template <typename R>
struct KernelVal {
  cplx<R> G, Fg;
};

// FP64 sine and cosine for |x| < 2^30: Cody-Waite reduction by pi/2 (two-part
// constant, fused multiply-add keeps the first subtraction exact) and the
// Taylor series of sin and cos on |r| <= pi/4, truncated after r^17 / r^18
// (truncation error below 1e-19).  Constants: pi/2 rounded to double and its
// remainder; 1/n! rounded to double.
__device__ __forceinline__ void sincos_taylor(double x, double* sn, double* cs) {
  const double PIO2_HI = 1.5707963267948966, PIO2_LO = 6.123233995736766e-17, TWO_OVER_PI = 0.6366197723675814;
  const double q = rint(x * TWO_OVER_PI);
  double r = fma(-q, PIO2_HI, x);
  r = fma(-q, PIO2_LO, r);
  const double r2 = r * r;
  // sin r = r + r^3 P(r^2),  P = -1/3! + r^2/5! - r^4/7! + ... + r^14/17!
  double ps = 2.8114572543455206e-15;           //  1/17!
  ps = fma(ps, r2, -7.647163731819816e-13);     // -1/15!
  ps = fma(ps, r2, 1.6059043836821613e-10);     //  1/13!
  ps = fma(ps, r2, -2.505210838544172e-08);     // -1/11!
  ps = fma(ps, r2, 2.755731922398589e-06);      //  1/9!
  ps = fma(ps, r2, -1.984126984126984e-04);     // -1/7!
  ps = fma(ps, r2, 8.333333333333333e-03);      //  1/5!
  ps = fma(ps, r2, -0.16666666666666666);       // -1/3!
  const double sr = fma(ps * r2, r, r);
  // cos r = 1 - r^2 Q(r^2),  Q = 1/2! - r^2/4! + r^4/6! - ... + r^16/18!
  double pc = 1.5619206968586225e-16;           //  1/18!
  pc = fma(pc, r2, -4.779477332387385e-14);     // -1/16!
  pc = fma(pc, r2, 1.1470745597729725e-11);     //  1/14!
  pc = fma(pc, r2, -2.08767569878681e-09);      // -1/12!
  pc = fma(pc, r2, 2.755731922398589e-07);      //  1/10!
  pc = fma(pc, r2, -2.48015873015873e-05);      // -1/8!
  pc = fma(pc, r2, 1.388888888888889e-03);      //  1/6!
  pc = fma(pc, r2, -0.041666666666666664);      // -1/4!
  pc = fma(pc, r2, 0.5);                        //  1/2!
  const double cr = fma(-pc, r2, 1.0);
  const int n = int(int64_t(q) & 3);
  const double s0 = (n & 1) ? cr : sr, c0 = (n & 1) ? sr : cr;
  *sn = (n & 2) ? -s0 : s0;
  *cs = ((n + 1) & 2) ? -c0 : c0;
}

// FP64 exp(x) for -700 < x < 700: x = m ln2 + r, |r| <= ln2/2, Taylor series
// of exp r through r^13 (truncation below 1e-17), scaled by 2^m.
__device__ __forceinline__ double exp_taylor(double x) {
  const double LN2_HI = 0.6931471805599453, LN2_LO = 2.3190468138462996e-17, INV_LN2 = 1.4426950408889634;
  const double m = rint(x * INV_LN2);
  double r = fma(-m, LN2_HI, x);
  r = fma(-m, LN2_LO, r);
  double p = 1.6059043836821613e-10;  // 1/13!
  p = fma(p, r, 2.08767569878681e-09);
  p = fma(p, r, 2.505210838544172e-08);
  p = fma(p, r, 2.755731922398589e-07);
  p = fma(p, r, 2.755731922398589e-06);
  p = fma(p, r, 2.48015873015873e-05);
  p = fma(p, r, 1.984126984126984e-04);
  p = fma(p, r, 1.388888888888889e-03);
  p = fma(p, r, 8.333333333333333e-03);
  p = fma(p, r, 0.041666666666666664);
  p = fma(p, r, 0.16666666666666666);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, int(m));
}

__device__ __forceinline__ void sincos_r(double x, double* s, double* c) { sincos_taylor(x, s, c); }
__device__ __forceinline__ void sincos_r(float x, float* s, float* c) { __sincosf(x, s, c); }
__device__ __forceinline__ double exp_r(double x) { return exp_taylor(x); }
__device__ __forceinline__ float exp_r(float x) { return __expf(x); }
__device__ __forceinline__ double rsqrt_r(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float rsqrt_r(float x) { return __frsqrt_rn(x); }

template <typename R>
__device__ __forceinline__ KernelVal<R> helmholtz(R r2, R kr, R ki, bool decay, R w) {
  R ir = rsqrt_r(r2);
  R r = r2 * ir;
  R s, c;
  sincos_r(kr * r, &s, &c);
  R amp = w * ir * R(INV_FOUR_PI);
  if (decay) amp *= exp_r(-ki * r);
  KernelVal<R> o;
  o.G = {amp * c, amp * s};
  // (ikr - 1) = (-ki r - 1) + i kr r
  R ar = -ki * r - R(1), ai = kr * r;
  R ir2 = ir * ir;
  o.Fg = {(o.G.re * ar - o.G.im * ai) * ir2, (o.G.re * ai + o.G.im * ar) * ir2};
  return o;
}

// Moments of one triangle pair at one wavenumber (coordinates relative to a
// local origin):  M0 = sum wG, Mx = sum wG x, My = sum wG y, Mxy = sum wG x.y,
// Nd = sum wFg (x - y), Nx = sum wFg (x cross y).
template <typename R>
struct Moments {
  cplx<R> M0, Mxy;
  cplx<R> Mx[3], My[3];
  cplx<R> Nd[3], Nx[3];
  __device__ __forceinline__ void zero() {
    M0 = {0, 0};
    Mxy = {0, 0};
    for (int d = 0; d < 3; ++d) Mx[d] = My[d] = Nd[d] = Nx[d] = {0, 0};
  }
  __device__ __forceinline__ void add(const KernelVal<R>& k, const R x[3], const R y[3], bool withC) {
    M0.re += k.G.re;
    M0.im += k.G.im;
    R xy = x[0] * y[0] + x[1] * y[1] + x[2] * y[2];
    Mxy.re += k.G.re * xy;
    Mxy.im += k.G.im * xy;
    for (int d = 0; d < 3; ++d) {
      Mx[d].re += k.G.re * x[d];
      Mx[d].im += k.G.im * x[d];
      My[d].re += k.G.re * y[d];
      My[d].im += k.G.im * y[d];
    }
    if (withC) {
      R cx[3] = {x[1] * y[2] - x[2] * y[1], x[2] * y[0] - x[0] * y[2], x[0] * y[1] - x[1] * y[0]};
      for (int d = 0; d < 3; ++d) {
        R dd = x[d] - y[d];
        Nd[d].re += k.Fg.re * dd;
        Nd[d].im += k.Fg.im * dd;
        Nx[d].re += k.Fg.re * cx[d];
        Nx[d].im += k.Fg.im * cx[d];
      }
    }
  }
};

// Contract moments against two RT0 fields u = a1 x - w1 (test) and
// v = a2 y - w2 (trial):
//   Sv = int int G u.v,  Sd = int int G div u div v,
//   Cc = -int int grad_x G . (v x u)
//      = -[(a1 w2 - a2 w1) . Nx + (w2 x w1) . Nd].
// S = -ik Sv - Sd/(ik).
template <typename R, typename A>
__device__ __forceinline__ void contract(const Moments<R>& m, A a1, const A w1[3], A a2, const A w2[3],
                                         double kr, double ki, bool withC, cplx<double>& S,
                                         cplx<double>& C) {
  double ww = double(w1[0]) * w2[0] + double(w1[1]) * w2[1] + double(w1[2]) * w2[2];
  double w2Mx_re = 0, w2Mx_im = 0, w1My_re = 0, w1My_im = 0;
  for (int d = 0; d < 3; ++d) {
    w2Mx_re += double(w2[d]) * m.Mx[d].re;
    w2Mx_im += double(w2[d]) * m.Mx[d].im;
    w1My_re += double(w1[d]) * m.My[d].re;
    w1My_im += double(w1[d]) * m.My[d].im;
  }
  double aa = double(a1) * a2;
  double sv_re = aa * m.Mxy.re - double(a1) * w2Mx_re - double(a2) * w1My_re + ww * m.M0.re;
  double sv_im = aa * m.Mxy.im - double(a1) * w2Mx_im - double(a2) * w1My_im + ww * m.M0.im;
  double sd_re = 4.0 * aa * m.M0.re, sd_im = 4.0 * aa * m.M0.im;
  // -ik Sv = (ki - i kr) Sv ; -1/(ik) Sd = i Sd / k = i Sd conj(k)/|k|^2
  double k2 = kr * kr + ki * ki;
  double t_re = (sd_re * kr + sd_im * ki) / k2;   // Sd conj(k)/|k|^2 (real part)
  double t_im = (sd_im * kr - sd_re * ki) / k2;
  S.re = ki * sv_re + kr * sv_im - t_im;
  S.im = ki * sv_im - kr * sv_re + t_re;
  if (withC) {
    double c_re = 0, c_im = 0;
    double wx[3] = {double(w2[1]) * w1[2] - double(w2[2]) * w1[1], double(w2[2]) * w1[0] - double(w2[0]) * w1[2],
                    double(w2[0]) * w1[1] - double(w2[1]) * w1[0]};
    for (int d = 0; d < 3; ++d) {
      double u = double(a1) * w2[d] - double(a2) * w1[d];
      c_re += u * m.Nx[d].re + wx[d] * m.Nd[d].re;
      c_im += u * m.Nx[d].im + wx[d] * m.Nd[d].im;
    }
    C.re = -c_re;
    C.im = -c_im;
  } else {
    C.re = C.im = 0;
  }
}

// Vertex order for a pair that shares nc >= 1 vertices: the shared vertices
// first, in the test triangle's order, then the remaining ones in ascending
// local order.  Returned as 2-bit local indices packed into oa / ob (slot v
// at bits 2v), computed with static indexing only so that everything stays
// in registers.
__device__ __forceinline__ int shared_order(const int va[3], const int vb[3], int& oa, int& ob) {
  int jb[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    int jj = -1;
#pragma unroll
    for (int j = 0; j < 3; ++j) jj = (va[i] == vb[j]) ? j : jj;
    jb[i] = jj;
  }
  int pos = 0;
  oa = 0;
  ob = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
    if (jb[i] >= 0) {
      oa |= i << (2 * pos);
      ob |= jb[i] << (2 * pos);
      ++pos;
    }
  const int nc = pos;
#pragma unroll
  for (int i = 0; i < 3; ++i)
    if (jb[i] < 0) {
      oa |= i << (2 * pos);
      ++pos;
    }
  pos = nc;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const bool sh = (va[0] == vb[j]) || (va[1] == vb[j]) || (va[2] == vb[j]);
    if (!sh) {
      ob |= j << (2 * pos);
      ++pos;
    }
  }
  return nc;
}

template <typename T>
__device__ __forceinline__ T pick3(const T v[3], int i) { return i == 0 ? v[0] : (i == 1 ? v[1] : v[2]); }

// The same contraction with all arithmetic in R (FP32 for FP32 operators,
// whose entries are stored in FP32 anyway).
template <typename R>
__device__ __forceinline__ void contract_r(const Moments<R>& m, R a1, const R w1[3], R a2, const R w2[3], R kr, R ki,
                                           cplx<R>& S, cplx<R>& C) {
  const R ww = w1[0] * w2[0] + w1[1] * w2[1] + w1[2] * w2[2];
  R w2Mx_re = 0, w2Mx_im = 0, w1My_re = 0, w1My_im = 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    w2Mx_re += w2[d] * m.Mx[d].re;
    w2Mx_im += w2[d] * m.Mx[d].im;
    w1My_re += w1[d] * m.My[d].re;
    w1My_im += w1[d] * m.My[d].im;
  }
  const R aa = a1 * a2;
  const R sv_re = aa * m.Mxy.re - a1 * w2Mx_re - a2 * w1My_re + ww * m.M0.re;
  const R sv_im = aa * m.Mxy.im - a1 * w2Mx_im - a2 * w1My_im + ww * m.M0.im;
  const R sd_re = R(4) * aa * m.M0.re, sd_im = R(4) * aa * m.M0.im;
  const R ik2 = R(1) / (kr * kr + ki * ki);
  const R t_re = (sd_re * kr + sd_im * ki) * ik2, t_im = (sd_im * kr - sd_re * ki) * ik2;
  S.re = ki * sv_re + kr * sv_im - t_im;
  S.im = ki * sv_im - kr * sv_re + t_re;
  const R wx[3] = {w2[1] * w1[2] - w2[2] * w1[1], w2[2] * w1[0] - w2[0] * w1[2], w2[0] * w1[1] - w2[1] * w1[0]};
  R c_re = 0, c_im = 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const R u = a1 * w2[d] - a2 * w1[d];
    c_re += u * m.Nx[d].re + wx[d] * m.Nd[d].re;
    c_im += u * m.Nx[d].im + wx[d] * m.Nd[d].im;
  }
  C.re = -c_re;
  C.im = -c_im;
}

template <typename T>
__device__ __forceinline__ void atomic_add(T* p, T v) {
  unsafeAtomicAdd(p, v);
}

}  // namespace pmchwt
