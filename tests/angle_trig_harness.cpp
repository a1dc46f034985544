// CPU check of sincos_angle against the C library's double sin and cos: every
// float angle on a dense grid of [-lim, lim], the quadrant boundaries k pi/2
// and their float neighbours, and tiny angles.  Prints "ok" and the largest
// error in units of 2^-24 (half an FP32 ulp of 1), or the first failure.
#define __host__
#define __device__
#include "angle_trig.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>

int main(int argc, char** argv) {
  const double lim = argc > 1 ? atof(argv[1]) : 100.0;
  const double bound = argc > 2 ? atof(argv[2]) : 4.0;  // largest error allowed, in 2^-24
  const double unit = std::ldexp(1.0, -24);
  double worst = 0.0;
  float worst_t = 0.0f;
  auto check = [&](float t) {
    float s, c;
    optmi::sincos_angle(t, &s, &c);
    const double es = std::fabs((double)s - std::sin((double)t)) / unit;
    const double ec = std::fabs((double)c - std::cos((double)t)) / unit;
    const double e = es > ec ? es : ec;
    if (!(e <= bound)) {
      printf("FAIL t=%.9g sin %.9g (%.17g) cos %.9g (%.17g) err %.3g\n", t, s, std::sin((double)t), c,
             std::cos((double)t), e);
      exit(1);
    }
    if (e > worst) {
      worst = e;
      worst_t = t;
    }
  };
  const int n = 4000000;
  for (int i = 0; i <= n; ++i) check((float)(-lim + 2.0 * lim * i / n));
  for (int k = -(int)(lim / 1.5707963267948966); k <= (int)(lim / 1.5707963267948966); ++k) {
    const float t = (float)(k * 1.5707963267948966);
    check(t);
    check(std::nextafter(t, 1e30f));
    check(std::nextafter(t, -1e30f));
    for (int j = 1; j < 64; ++j) check((float)(k * 1.5707963267948966 + 0.7853981633974483 * j / 64.0));
  }
  for (float t = 1e-30f; t < 1.0f; t *= 1.37f) {
    check(t);
    check(-t);
  }
  check(0.0f);
  printf("ok %.3f at t=%.9g\n", worst, worst_t);
  return 0;
}
