// Host build of the shared device header's field-coefficient functions, for CPU tests.
// Reads lines "<fn> <args...>" from stdin and prints the results with 17 digits.
#include <cstdio>
#include <cstring>

#include "drt_geom.h"

using namespace drt;

int main() {
  char fn[32];
  while (std::scanf("%31s", fn) == 1) {
    if (!std::strcmp(fn, "F64") || !std::strcmp(fn, "F32")) {
      double X;
      std::scanf("%lf", &X);
      if (fn[1] == '6') {
        Cx<double> v = utd_transition<double>(X);
        std::printf("%.17g %.17g\n", v.re, v.im);
      } else {
        Cx<float> v = utd_transition<float>(float(X));
        std::printf("%.9g %.9g\n", v.re, v.im);
      }
    } else if (!std::strcmp(fn, "D64")) {
      double phi, php, sb, n, k, Ld;
      int pol;
      std::scanf("%lf %lf %lf %lf %lf %lf %d", &phi, &php, &sb, &n, &k, &Ld, &pol);
      Cx<double> v = utd_coefficient<double, double>(phi, php, sb, n, k, Ld, pol);
      std::printf("%.17g %.17g\n", v.re, v.im);
    } else if (!std::strcmp(fn, "D32")) {   // binary64 angles, binary32 field arithmetic
      double phi, php, sb, n, k, Ld;
      int pol;
      std::scanf("%lf %lf %lf %lf %lf %lf %d", &phi, &php, &sb, &n, &k, &Ld, &pol);
      Cx<float> v = utd_coefficient<double, float>(phi, php, float(sb), n, float(k), float(Ld), pol);
      std::printf("%.9g %.9g\n", v.re, v.im);
    } else if (!std::strcmp(fn, "G64")) {
      double ct, er, sg, lam;
      int pec, pol;
      std::scanf("%lf %lf %lf %lf %d %d", &ct, &er, &sg, &lam, &pec, &pol);
      DMat m{er, sg, pec, 0};
      Cx<double> v = fresnel<double>(ct, m, lam, pol);
      std::printf("%.17g %.17g\n", v.re, v.im);
    } else if (!std::strcmp(fn, "SC32")) {   // binary32 sin / cos of a bounded argument
      double x;
      std::scanf("%lf", &x);
      float s, c;
      sincos_small(float(x), s, c);
      std::printf("%.9g %.9g\n", s, c);
    } else if (!std::strcmp(fn, "G32")) {
      double ct, er, sg, lam;
      int pec, pol;
      std::scanf("%lf %lf %lf %lf %d %d", &ct, &er, &sg, &lam, &pec, &pol);
      DMat m{er, sg, pec, 0};
      Cx<float> v = fresnel<float>(float(ct), m, float(lam), pol);
      std::printf("%.9g %.9g\n", v.re, v.im);
    } else if (!std::strcmp(fn, "ER64")) {
      int alpha;
      double ct;
      std::scanf("%d %lf", &alpha, &ct);
      std::printf("%.17g\n", er_norm_directive<double>(alpha, ct));
    }
  }
  return 0;
}
