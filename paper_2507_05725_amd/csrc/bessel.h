// FP64 Bessel functions of order zero for real z >= 0, for the Helmholtz
// fundamental solution Phi_k(r) = (i/4) H0^(1)(k r) = (i/4)(J0 + i Y0),
// written from published mathematics (no vendor math library internals):
//
//   z < 4        the ascending series in u = z^2/4 (DLMF 10.8.1, 10.8.2),
//                17 terms, for J0 and for the regular part Y0hat below
//   z >= 4       the modulus-phase form of Hankel's expansion (DLMF 10.17.3,
//                10.17.4) with the exact modulus functions P(z), Q(z) in
//                place of their divergent series: polynomial fits in
//                (4/z)^2 on [4, 8), in (8/z)^2 on [8, 24) and in (24/z)^2
//                beyond (bessel_fit.h, written by bessel_fit.py), phase by
//                sin/cos of z.
//
// Besides J0 and Y0 the routines expose the regular part
//   Y0hat(z) = Y0(z) - (2/pi)(log(z/2) + gamma) J0(z),
// an entire function of z^2 that the Nystrom assembly needs near the
// diagonal without cancellation.  Host-compiled copies of these routines
// are checked against mpmath over the full argument range of the workloads.
//
// Order one (the double-layer kernel of closed curves) keeps Miller's
// backward recurrence below z = 16.5 and Hankel's series above (bessel_01).
#pragma once

#include "bessel_fit.h"
#include "common.h"

namespace fthms {

struct HankelAsymCoef {
  double p[14];  // (-1)^k a_{2k}(0)
  double q[14];  // (-1)^k a_{2k+1}(0)
};

// a_k(0) = prod_{j=1..k} (-(2j-1)^2) / (k! 8^k)   (DLMF 10.17.1 at nu = 0)
constexpr HankelAsymCoef make_hankel_asym_coef() {
  HankelAsymCoef c{};
  double a[28] = {};
  a[0] = 1.0;
  for (int k = 1; k < 28; ++k)
    a[k] = a[k - 1] * (-(double)((2 * k - 1) * (2 * k - 1))) / (8.0 * k);
  for (int k = 0; k < 14; ++k) {
    c.p[k] = ((k & 1) ? -1.0 : 1.0) * a[2 * k];
    c.q[k] = ((k & 1) ? -1.0 : 1.0) * a[2 * k + 1];
  }
  return c;
}

// J0 and Y0 from Hankel's expansion, phase via sin/cos of z itself:
// cos(z - pi/4) = (cos z + sin z)/sqrt2, sin(z - pi/4) = (sin z - cos z)/sqrt2.
FTHMS_HD void bessel_asym(double z, double &j0, double &y0) {
  constexpr HankelAsymCoef c = make_hankel_asym_coef();
  const double iz = 1.0 / z;
  const double w = iz * iz;
  double P = c.p[13], Q = c.q[13];
#pragma unroll
  for (int k = 12; k >= 0; --k) {
    P = P * w + c.p[k];
    Q = Q * w + c.q[k];
  }
  Q *= iz;
  double s, co;
  sincos(z, &s, &co);
  const double r2 = 0.70710678118654752440084436210484904;
  const double cm = (co + s) * r2, sm = (s - co) * r2;
  const double f = sqrt((2.0 / kPi) * iz);
  j0 = f * (P * cm - Q * sm);
  y0 = f * (P * sm + Q * cm);
}

constexpr double kBesselAsymFrom = 16.5;

// (2/pi)(log(z/2) + gamma): the log part separating Y0 from Y0hat
FTHMS_HD double bessel_logpart(double z) {
  return (2.0 / kPi) * (log(0.5 * z) + kEulerGamma);
}

// Region boundaries of the order-zero routines.
constexpr double kBesselSeriesTo = 4.0, kBesselMidTo = 8.0;

// J0 and Y0hat for z < 4 by the ascending series.
FTHMS_HD void bessel_series(double z, double &j0, double &y0hat) {
  const double u = 0.25 * z * z;
  double a = kSeriesJ[16], b = kSeriesY[16];
#pragma unroll
  for (int k = 15; k >= 0; --k) {
    a = a * u + kSeriesJ[k];
    b = b * u + kSeriesY[k];
  }
  j0 = a;
  y0hat = b;
}

// sin x and cos x for the phases of Hankel's expansion (|x| below 1e6):
// Cody and Waite's argument reduction x = n pi/2 + r, |r| <= pi/4, with
// pi/2 split into two doubles and fused multiply-adds (each product exact
// before its one rounding: r within 6e-17 of its value), then the Taylor
// series of sin r through r^17 and of cos r through r^16 (the first omitted
// terms below 1e-16 of one on |r| <= pi/4) and the quadrant n mod 4.
// Larger arguments take the library's sincos.
FTHMS_HD void phase_sincos(double x, double &s, double &c) {
  if (!(fabs(x) < 1e6)) {
    sincos(x, &s, &c);
    return;
  }
  const double n = rint(x * 0.63661977236758138);  // 2 / pi
  double r = fma(-n, 1.5707963267948966, x);
  r = fma(-n, 6.123233995736766e-17, r);
  const double u = r * r;
  // 1 / k! for k = 2 .. 17
  double sp = fma(u, 2.8114572543455206e-15, -7.647163731819816e-13);
  sp = fma(u, sp, 1.6059043836821613e-10);
  sp = fma(u, sp, -2.505210838544172e-08);
  sp = fma(u, sp, 2.7557319223985893e-06);
  sp = fma(u, sp, -0.0001984126984126984);
  sp = fma(u, sp, 0.008333333333333333);
  sp = fma(u, sp, -0.16666666666666666);
  sp = fma(u * r, sp, r);
  double cp = fma(u, 4.779477332387385e-14, -1.1470745597729725e-11);
  cp = fma(u, cp, 2.08767569878681e-09);
  cp = fma(u, cp, -2.755731922398589e-07);
  cp = fma(u, cp, 2.48015873015873e-05);
  cp = fma(u, cp, -0.001388888888888889);
  cp = fma(u, cp, 0.041666666666666664);
  cp = fma(u, cp, -0.5);
  cp = fma(u, cp, 1.0);
  const int q = (int)n & 3;
  const double a = (q & 1) ? cp : sp, b = (q & 1) ? sp : cp;  // sin, cos up to sign
  s = (q & 2) ? -a : a;
  c = ((q + 1) & 2) ? -b : b;
}

// The modulus functions P(z) and Q(z) for z >= 4 (iz = 1/z).
FTHMS_HD void bessel_pq(double z, double iz, double &P, double &Q) {
  double Qz;
  if (z < kBesselMidTo) {
    const double x = (16.0 * iz * iz - kPQMidC) * (1.0 / kPQMidH);
    P = kPQMidP[14];
    Qz = kPQMidQ[14];
#pragma unroll
    for (int k = 13; k >= 0; --k) {
      P = P * x + kPQMidP[k];
      Qz = Qz * x + kPQMidQ[k];
    }
  } else if (z < kPQFarZ) {
    const double w = 64.0 * iz * iz;
    P = kPQBigP[12];
    Qz = kPQBigQ[12];
#pragma unroll
    for (int k = 11; k >= 0; --k) {
      P = P * w + kPQBigP[k];
      Qz = Qz * w + kPQBigQ[k];
    }
  } else {
    const double v = (kPQFarZ * kPQFarZ) * iz * iz;
    P = kPQFarP[6];
    Qz = kPQFarQ[6];
#pragma unroll
    for (int k = 5; k >= 0; --k) {
      P = P * v + kPQFarP[k];
      Qz = Qz * v + kPQFarQ[k];
    }
  }
  Q = Qz * iz;
}

// J0 = f (P cos chi - Q sin chi), Y0 = f (P sin chi + Q cos chi), chi =
// z - pi/4, from cos z and sin z and the amplitude f = sqrt(2/(pi z)):
// cos(z - pi/4) = (cos z + sin z)/sqrt2, sin(z - pi/4) = (sin z - cos z)/sqrt2.
FTHMS_HD void bessel_combine(double P, double Q, double cz, double sz, double f, double &j0,
                             double &y0) {
  const double r2 = 0.70710678118654752440084436210484904;
  const double cm = (cz + sz) * r2, sm = (sz - cz) * r2;
  j0 = f * (P * cm - Q * sm);
  y0 = f * (P * sm + Q * cm);
}

// The same polynomials with their coefficients read from a table (pairs
// (J, Y) / (P, zQ) in one double2 each, in the order of bessel_fit.h):
// kernels that loop over wavenumbers keep the 52 pairs in LDS instead of in
// registers.  Same operations in the same order as bessel_series and
// bessel_pq, so the results are identical.
constexpr int kBesselTabSeries = 0, kBesselTabMid = 17, kBesselTabBig = 32, kBesselTabFar = 45,
              kBesselTabLen = 52;

FTHMS_HD void bessel_tab_fill(double2 *tab, int i) {
  if (i < 17) tab[kBesselTabSeries + i] = make_double2(kSeriesJ[i], kSeriesY[i]);
  else if (i < 32) tab[i] = make_double2(kPQMidP[i - 17], kPQMidQ[i - 17]);
  else if (i < 45) tab[i] = make_double2(kPQBigP[i - 32], kPQBigQ[i - 32]);
  else if (i < 52) tab[i] = make_double2(kPQFarP[i - 45], kPQFarQ[i - 45]);
}

__device__ __forceinline__ void bessel_series_tab(double z, const double2 *tab, double &j0,
                                                  double &y0hat) {
  const double u = 0.25 * z * z;
  const double2 *c = tab + kBesselTabSeries;
  double a = c[16].x, b = c[16].y;
#pragma unroll
  for (int k = 15; k >= 0; --k) {
    const double2 ck = c[k];
    a = a * u + ck.x;
    b = b * u + ck.y;
  }
  j0 = a;
  y0hat = b;
}

__device__ __forceinline__ void bessel_pq_tab(double z, double iz, const double2 *tab, double &P,
                                              double &Q) {
  double Qz;
  if (z < kBesselMidTo) {
    const double x = (16.0 * iz * iz - kPQMidC) * (1.0 / kPQMidH);
    const double2 *c = tab + kBesselTabMid;
    P = c[14].x;
    Qz = c[14].y;
#pragma unroll
    for (int k = 13; k >= 0; --k) {
      const double2 ck = c[k];
      P = P * x + ck.x;
      Qz = Qz * x + ck.y;
    }
  } else if (z < kPQFarZ) {
    const double w = 64.0 * iz * iz;
    const double2 *c = tab + kBesselTabBig;
    P = c[12].x;
    Qz = c[12].y;
#pragma unroll
    for (int k = 11; k >= 0; --k) {
      const double2 ck = c[k];
      P = P * w + ck.x;
      Qz = Qz * w + ck.y;
    }
  } else {
    const double v = (kPQFarZ * kPQFarZ) * iz * iz;
    const double2 *c = tab + kBesselTabFar;
    P = c[6].x;
    Qz = c[6].y;
#pragma unroll
    for (int k = 5; k >= 0; --k) {
      const double2 ck = c[k];
      P = P * v + ck.x;
      Qz = Qz * v + ck.y;
    }
  }
  Q = Qz * iz;
}

// J0 and Y0 for z >= 4 from the fitted modulus functions, the phase from
// sin/cos of z itself.
FTHMS_HD void bessel_modphase(double z, double &j0, double &y0) {
  const double iz = 1.0 / z;
  double P, Q;
  bessel_pq(z, iz, P, Q);
  double s, co;
  phase_sincos(z, s, co);
  bessel_combine(P, Q, co, s, sqrt((2.0 / kPi) * iz), j0, y0);
}

// J0(z) and Y0hat(z), z >= 0.
FTHMS_HD void bessel_j0_y0hat(double z, double &j0, double &yh) {
  if (z < kBesselSeriesTo) {
    bessel_series(z, j0, yh);
  } else {
    double y0;
    bessel_modphase(z, j0, y0);
    yh = y0 - bessel_logpart(z) * j0;
  }
}

// J0(z) and Y0(z), z > 0.
FTHMS_HD void bessel_j0_y0(double z, double &j0, double &y0) {
  if (z < kBesselSeriesTo) {
    double yh;
    bessel_series(z, j0, yh);
    y0 = yh + bessel_logpart(z) * j0;
  } else {
    bessel_modphase(z, j0, y0);
  }
}

// ---- order one (the double-layer kernel of closed curves) ----------------
//
//   z < 1e-6     leading terms: J1 = z/2, Y1 = -2/(pi z) + (z/pi)(log(z/2)
//                + gamma - 1/2)  (DLMF 10.8.1, 10.8.2 at n = 1)
//   z < 16.5     the same backward recurrence; J1 from it, and
//                Y1 = -Y0' = -(2/(pi z)) J0 + (2/pi)(log(z/2) + gamma) J1
//                     + (2/pi) sum_k (-1)^k (J_{2k-1} - J_{2k+1}) / k
//                (differentiating the Neumann series of Y0 term by term with
//                J_n' = (J_{n-1} - J_{n+1})/2), summed as sum_k c_k J_{2k-1},
//                c_1 = -1, c_k = (-1)^k (2k - 1) / (k (k - 1))
//   z >= 16.5    Hankel's expansion at nu = 1 (DLMF 10.17.3, 10.17.4).

// a_k(1) = prod_{j=1..k} (4 - (2j-1)^2) / (k! 8^k)   (DLMF 10.17.1 at nu = 1)
constexpr HankelAsymCoef make_hankel_asym_coef1() {
  HankelAsymCoef c{};
  double a[28] = {};
  a[0] = 1.0;
  for (int k = 1; k < 28; ++k)
    a[k] = a[k - 1] * (4.0 - (double)((2 * k - 1) * (2 * k - 1))) / (8.0 * k);
  for (int k = 0; k < 14; ++k) {
    c.p[k] = ((k & 1) ? -1.0 : 1.0) * a[2 * k];
    c.q[k] = ((k & 1) ? -1.0 : 1.0) * a[2 * k + 1];
  }
  return c;
}

template <int NS>
FTHMS_HD void bessel_miller01(double z, double &j0, double &j1, double &y0, double &y1) {
  const double rz = 2.0 / z;
  double jp1 = 0.0, jn = 1.0e-250, even = 0.0, neu = 0.0, odd = 0.0, j1u = 0.0;
#pragma unroll
  for (int n = NS; n >= 1; --n) {
    const double jm1 = ((double)n * rz) * jn - jp1;
    jp1 = jn;
    jn = jm1;  // J_{n-1}, unnormalised
    const int m = n - 1;
    if (m > 0 && (m & 1) == 0) {
      const int k = m >> 1;
      even += jn;
      neu += (((k & 1) ? -1.0 : 1.0) / (double)k) * jn;
    }
    if (m & 1) {
      const int k = (m + 1) >> 1;  // m = 2k - 1
      const double ck = (k == 1) ? -1.0
                                 : ((k & 1) ? -1.0 : 1.0) * (double)(2 * k - 1) /
                                       ((double)k * (double)(k - 1));
      odd += ck * jn;
      if (m == 1) j1u = jn;
    }
  }
  const double inv = 1.0 / (jn + 2.0 * even);
  j0 = jn * inv;
  j1 = j1u * inv;
  const double lp = bessel_logpart(z);
  y0 = lp * j0 - (4.0 / kPi) * neu * inv;
  y1 = -(2.0 / kPi) * j0 / z + lp * j1 + (2.0 / kPi) * odd * inv;
}

// J1 and Y1 from Hankel's expansion, phase z - 3pi/4:
// cos(z - 3pi/4) = (sin z - cos z)/sqrt2, sin(z - 3pi/4) = -(sin z + cos z)/sqrt2.
FTHMS_HD void bessel_asym1(double z, double &j1, double &y1) {
  constexpr HankelAsymCoef c = make_hankel_asym_coef1();
  const double iz = 1.0 / z;
  const double w = iz * iz;
  double P = c.p[13], Q = c.q[13];
#pragma unroll
  for (int k = 12; k >= 0; --k) {
    P = P * w + c.p[k];
    Q = Q * w + c.q[k];
  }
  Q *= iz;
  double s, co;
  sincos(z, &s, &co);
  const double r2 = 0.70710678118654752440084436210484904;
  const double cm = (s - co) * r2, sm = -(s + co) * r2;
  const double f = sqrt((2.0 / kPi) * iz);
  j1 = f * (P * cm - Q * sm);
  y1 = f * (P * sm + Q * cm);
}

// J0, Y0, J1, Y1 at z > 0.
FTHMS_HD void bessel_01(double z, double &j0, double &y0, double &j1, double &y1) {
  if (z < 1.0e-6) {
    const double q = 0.25 * z * z;
    j0 = 1.0 - q;
    y0 = bessel_logpart(z) * j0 + (2.0 / kPi) * q;
    j1 = 0.5 * z;
    y1 = -(2.0 / kPi) / z + (z / kPi) * (log(0.5 * z) + kEulerGamma - 0.5);
  } else if (z < 8.0) {
    bessel_miller01<32>(z, j0, j1, y0, y1);
  } else if (z < kBesselAsymFrom) {
    bessel_miller01<48>(z, j0, j1, y0, y1);
  } else {
    bessel_asym(z, j0, y0);
    bessel_asym1(z, j1, y1);
  }
}

}  // namespace fthms
