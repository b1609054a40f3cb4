// Host-side probe of the device Bessel routines: reads z values on stdin,
// prints "z j0 y0 j0' y0hat j0'' y0'' j1 y1 sin cos" (the order-zero values
// from the order-zero routines, then from the combined order-0/1 routine,
// then the phase sine and cosine) with 17 significant digits.  Built by the test
// suite with hipcc; it runs on the CPU only and launches nothing.
#include <cstdio>
#include "../../paper_2507_05725_amd/csrc/bessel.h"

int main() {
  double z;
  while (std::scanf("%lf", &z) == 1) {
    double j0, y0, j0b, yh, j0c, y0c, j1, y1, sn, cs;
    fthms::phase_sincos(z, sn, cs);
    fthms::bessel_j0_y0(z, j0, y0);
    fthms::bessel_j0_y0hat(z, j0b, yh);
    fthms::bessel_01(z, j0c, y0c, j1, y1);
    std::printf("%.17g %.17g %.17g %.17g %.17g %.17g %.17g %.17g %.17g %.17g %.17g\n", z, j0, y0, j0b,
                yh, j0c, y0c, j1, y1, sn, cs);
  }
  return 0;
}
