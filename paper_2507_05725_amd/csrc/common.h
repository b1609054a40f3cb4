// Shared types and small helpers for the libfthms HIP sources (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define FTHMS_HD __host__ __device__ __forceinline__

namespace fthms {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kEulerGamma = 0.57721566490153286060651209008240243;

// Device memory one batched call keeps in flight for its matrices and their
// workspace (less under a context budget): 32 GiB of the 288 GB HBM, which
// holds the 4096 N = 512 matrices of a refined batch (about 26 GB) at once.
constexpr size_t kChunkBytes = (size_t)32 << 30;

template <typename T> struct cplx;
template <> struct cplx<double> { using type = double2; };
template <> struct cplx<float> { using type = float2; };
template <typename T> using cplx_t = typename cplx<T>::type;

template <typename T> FTHMS_HD cplx_t<T> mk(T re, T im) {
  cplx_t<T> z;
  z.x = re;
  z.y = im;
  return z;
}
FTHMS_HD double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
FTHMS_HD double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
FTHMS_HD double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a - b*c
FTHMS_HD double2 cfms(double2 a, double2 b, double2 c) {
  return make_double2(a.x - b.x * c.x + b.y * c.y, a.y - b.x * c.y - b.y * c.x);
}
// a + b*c
FTHMS_HD double2 cfma(double2 a, double2 b, double2 c) {
  return make_double2(a.x + b.x * c.x - b.y * c.y, a.y + b.x * c.y + b.y * c.x);
}
// 1 / a, scaled to avoid overflow for the magnitudes met here
FTHMS_HD double2 crcp(double2 a) {
  double s = fabs(a.x) > fabs(a.y) ? fabs(a.x) : fabs(a.y);
  double ar = a.x / s, ai = a.y / s;
  double d = s * (ar * ar + ai * ai);
  return make_double2(ar / d, -ai / d);
}
FTHMS_HD double cabs1(double2 a) { return fabs(a.x) + fabs(a.y); }
FTHMS_HD double cnorm2(double2 a) { return a.x * a.x + a.y * a.y; }

FTHMS_HD double2 to_d2(double2 a) { return a; }
FTHMS_HD double2 to_d2(float2 a) { return make_double2((double)a.x, (double)a.y); }
template <typename T> FTHMS_HD cplx_t<T> from_d2(double2 a);
template <> FTHMS_HD double2 from_d2<double>(double2 a) { return a; }
template <> FTHMS_HD float2 from_d2<float>(double2 a) {
  return make_float2((float)a.x, (float)a.y);
}

}  // namespace fthms
