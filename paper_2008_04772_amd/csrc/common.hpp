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

__device__ __forceinline__ void sincos_r(double x, double* s, double* c) { sincos(x, s, c); }
__device__ __forceinline__ void sincos_r(float x, float* s, float* c) { __sincosf(x, s, c); }
__device__ __forceinline__ double exp_r(double x) { return exp(x); }
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

template <typename T>
__device__ __forceinline__ void atomic_add(T* p, T v) {
  unsafeAtomicAdd(p, v);
}

}  // namespace pmchwt
