// FP64 exponential and sine/cosine for the bounded arguments of the kernel
// exp(-s r) (r at most a few surface diameters, Re s > 0).
//
// Published methods (Cody & Waite, "Software Manual for the Elementary
// Functions", 1980): additive argument reduction by a multi-part constant so
// that k*C_hi is exact, then a truncated Taylor series on the reduced
// interval, evaluated by Horner's rule with fused multiply-adds.
//   exp:    x = k ln2 + r, |r| <= ln2/2, degree 13 (truncation < 5e-18 relative)
//   sincos: t = k pi/2 + r, |r| <= pi/4, degrees 17 / 18 (truncation < 1e-19)
// The split constants are ln2 and pi/2 cut into 32/33-bit leading parts and
// remainders (computed in extended precision); k*hi is exact for |k| < 2^20.
#pragma once
#include <hip/hip_runtime.h>

namespace cqm {

__device__ __forceinline__ double exp_nonpos(double x) {
  // x <= 0 expected; results below the normal range flush to zero
  if (x < -708.0) return 0.0;
  const double k = rint(x * 1.4426950408889634);
  double r = fma(-k, 0.6931471803691238, x);
  r = fma(-k, 1.9082149292705877e-10, r);
  double p = 1.6059043836821613e-10;  // 1/13!
  p = fma(p, r, 2.08767569878681e-09);   // 1/12!
  p = fma(p, r, 2.505210838544172e-08);  // 1/11!
  p = fma(p, r, 2.755731922398589e-07);  // 1/10!
  p = fma(p, r, 2.7557319223985893e-06); // 1/9!
  p = fma(p, r, 2.48015873015873e-05);   // 1/8!
  p = fma(p, r, 0.0001984126984126984);  // 1/7!
  p = fma(p, r, 0.001388888888888889);   // 1/6!
  p = fma(p, r, 0.008333333333333333);   // 1/5!
  p = fma(p, r, 0.041666666666666664);   // 1/4!
  p = fma(p, r, 0.16666666666666666);    // 1/3!
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, (int)k);
}

__device__ __forceinline__ void sincos_bounded(double t, double* s, double* c) {
  const double k = rint(t * 0.6366197723675814);
  double r = fma(-k, 1.5707963267341256, t);
  r = fma(-k, 6.077100506303966e-11, r);
  r = fma(-k, 2.0222662487959506e-21, r);
  const double r2 = r * r;
  // sin r = r (1 - r2/3! + r2^2/5! - ...), through r^17
  double ps = 2.8114572543455206e-15;        // 1/17!
  ps = fma(ps, r2, -7.647163731819816e-13);  // -1/15!
  ps = fma(ps, r2, 1.6059043836821613e-10);  // 1/13!
  ps = fma(ps, r2, -2.505210838544172e-08);  // -1/11!
  ps = fma(ps, r2, 2.7557319223985893e-06);  // 1/9!
  ps = fma(ps, r2, -0.0001984126984126984);  // -1/7!
  ps = fma(ps, r2, 0.008333333333333333);    // 1/5!
  ps = fma(ps, r2, -0.16666666666666666);    // -1/3!
  const double sr = fma(ps * r2, r, r);
  // cos r = 1 - r2/2! + r2^2/4! - ..., through r^18
  double pc = -1.5619206968586225e-16;       // -1/18!
  pc = fma(pc, r2, 4.779477332387385e-14);   // 1/16!
  pc = fma(pc, r2, -1.1470745597729725e-11); // -1/14!
  pc = fma(pc, r2, 2.08767569878681e-09);    // 1/12!
  pc = fma(pc, r2, -2.755731922398589e-07);  // -1/10!
  pc = fma(pc, r2, 2.48015873015873e-05);    // 1/8!
  pc = fma(pc, r2, -0.001388888888888889);   // -1/6!
  pc = fma(pc, r2, 0.041666666666666664);    // 1/4!
  pc = fma(pc, r2, -0.5);                    // -1/2!
  const double cr = fma(pc, r2, 1.0);
  const int q = ((int)k) & 3;
  const double a = (q & 1) ? cr : sr;
  const double b = (q & 1) ? sr : cr;
  *s = (q & 2) ? -a : a;
  *c = ((q + 1) & 2) ? -b : b;
}

// Table-driven variants (Tang's method, "Table-driven implementation of the
// exponential function in IEEE floating-point arithmetic", ACM TOMS 1989,
// and the same idea for sine/cosine): reduce by a multiple of a table step,
// look the step's value up, and evaluate a short Taylor polynomial on the
// small remainder.  `tab` (in LDS, 16-byte aligned) holds 2^(j/256) for
// j = 0..255, then the pairs (sin, cos)(2 pi j/256) (kFp64TabLen doubles,
// filled on the host in extended precision).  The nearest integer k comes
// from adding 1.5 * 2^52 (its low 32 bits are then k in two's complement),
// which also gives k for the table index without a conversion; the step is
// split into a leading part of 35 bits (k * hi exact for |k| < 2^18) and a
// remainder.  Both functions are branch-free.
constexpr int kFp64TabLen = 768;
// A finer sine/cosine table, (sin, cos)(2 pi j/512) for j = 0..511, stored
// after the first one (the dense assembly stages the exponential part and
// this one): its remainder is half as large, so cos - 1 needs one Taylor
// term less.
constexpr int kFp64Tab512Off = 768, kFp64Tab512Len = 1024;
constexpr int kFp64TabTotal = kFp64Tab512Off + kFp64Tab512Len;
constexpr double kRoundMagic = 6755399441055744.0;  // 1.5 * 2^52

__device__ __forceinline__ double exp_tab(double x, const double* tab) {
  // x = (256 m + j) ln2/256 + r, |r| <= ln2/512; x below -708 is taken as
  // -708 (the result, 3.3e-308, stands for 0)
  const double xc = fmax(x, -708.0);
  const double kd = fma(xc, 369.3299304675746, kRoundMagic);  // 256/ln2
  const int ik = (int)__double_as_longlong(kd);
  const double k = kd - kRoundMagic;
  double r = fma(-k, 0.0027076061741126978, xc);
  r = fma(-k, -5.0411407304988844e-14, r);
  // exp r through r^4 (truncation < 4e-17 relative)
  double p = 0.041666666666666664;        // 1/4!
  p = fma(p, r, 0.16666666666666666);     // 1/3!
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(tab[ik & 255] * p, ik >> 8);
}

__device__ __forceinline__ void sincos_tab(double t, const double* tab, double* s, double* c) {
  // t = k 2pi/256 + r, |r| <= pi/256; (sin, cos)(2 pi k/256) from the table
  const double kd = fma(t, 40.74366543152521, kRoundMagic);  // 256/(2 pi)
  const int ik = (int)__double_as_longlong(kd);
  const double k = kd - kRoundMagic;
  double r = fma(-k, 0.024543692606130207, t);
  r = fma(-k, 4.005225236866436e-14, r);
  const double r2 = r * r;
  // sin r through r^5 (truncation < 1e-17 absolute), cos r - 1 through r^6
  // (truncation < 2e-20)
  double ps = 0.008333333333333333;           // 1/5!
  ps = fma(ps, r2, -0.16666666666666666);     // -1/3!
  const double sr = fma(ps * r2, r, r);
  double pc = -0.001388888888888889;          // -1/6!
  pc = fma(pc, r2, 0.041666666666666664);     // 1/4!
  pc = fma(pc, r2, -0.5);                     // -1/2!
  const double cm1 = pc * r2;
  const double2 sc = *reinterpret_cast<const double2*>(tab + 256 + 2 * (ik & 255));
  // sin(A + r) = sA + (sA (cos r - 1) + cA sin r), likewise cos(A + r)
  *s = fma(sc.y, sr, fma(sc.x, cm1, sc.x));
  *c = fma(-sc.x, sr, fma(sc.y, cm1, sc.y));
}

// The same functions for arguments given in table steps: u = x 256/ln2 for
// the exponential, u = t 512/(2 pi) for sine/cosine on the finer table (the
// caller scales the frequency once instead of every argument).  k = round(u)
// and the remainder f = u - k are exact, so no Cody-Waite split is needed;
// the Taylor coefficients carry the powers of the step (ln2/256, 2 pi/512).
// The rounding of u costs about |x| 2^-53 absolute in the argument, the same
// order as forming x = -Re(s) r itself.  exp_tabu requires u >= -708 256/ln2.
__device__ __forceinline__ double exp_tabu(double u, const double* tab) {
  constexpr double L = 0.0027076061740622863;  // ln2/256
  const double kd = u + kRoundMagic;
  const int ik = (int)__double_as_longlong(kd);
  const double f = u - (kd - kRoundMagic);  // |f| <= 1/2
  // exp(L f) through (L f)^4
  double p = L * L * L * L / 24.0;
  p = fma(p, f, L * L * L / 6.0);
  p = fma(p, f, L * L / 2.0);
  p = fma(p, f, L);
  p = fma(p, f, 1.0);
  return ldexp(tab[ik & 255] * p, ik >> 8);
}

// u in steps of 2 pi/512; tab512 is the 512-entry (sin, cos) table.
__device__ __forceinline__ void sincos_tabu512(double u, const double* tab512, double* s,
                                               double* c) {
  constexpr double A = 0.01227184630308513;  // 2 pi/512
  const double kd = u + kRoundMagic;
  const int ik = (int)__double_as_longlong(kd);
  const double f = u - (kd - kRoundMagic);  // |A f| <= pi/512
  const double f2 = f * f;
  // sin(A f) through (A f)^5; cos(A f) - 1 through (A f)^4 (the next term
  // is below 8e-17)
  double ps = A * A * A * A * A / 120.0;
  ps = fma(ps, f2, -A * A * A / 6.0);
  ps = fma(ps, f2, A);
  const double sr = ps * f;
  const double pc = fma(A * A * A * A / 24.0, f2, -A * A / 2.0);
  const double cm1 = pc * f2;
  const double2 sc = *reinterpret_cast<const double2*>(tab512 + 2 * (ik & 511));
  *s = fma(sc.y, sr, fma(sc.x, cm1, sc.x));
  *c = fma(-sc.x, sr, fma(sc.y, cm1, sc.y));
}


}  // namespace cqm
