// Host build of the step kernels' phase routines (the (cos(phi) - 1, sin(phi), sin(phi)/phi)
// helpers of the real-space exponential), for a CPU check against fp64 sine and cosine.  The
// routines are compiled from the same header the kernels use.
//
// Reads angles (one float per line, as hex float text) on stdin; prints for each: the angle, then
// cm1, s, sinc of the general (reduced) routine, then the same of the short routine, as hex floats.
#include <cstdio>
#include <cstdlib>

#include "fft_device.hpp"

int main() {
  char buf[128];
  while (std::fgets(buf, sizeof buf, stdin)) {
    const float phi = std::strtof(buf, nullptr);
    const sgpe::SinCosM1 r = sgpe::sincos_m1_reduced(phi);
    const sgpe::SinCosM1 s = sgpe::sincos_m1_small(phi);
    std::printf("%a %a %a %a %a %a %a\n", phi, r.cm1, r.s, r.sinc, s.cm1, s.s, s.sinc);
  }
  return 0;
}
