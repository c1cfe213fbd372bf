// Ray-sum records written by the geometry kernels and read by the ray-sum kernels.
#ifndef DRT_RECORDS_H
#define DRT_RECORDS_H

#include <hip/hip_runtime.h>

#include <cstdint>

namespace drt {

struct RecS { double L; float gr, gi, zr, zi; };       // split: 24 B
// split, MFMA path: 32 B.  Phases in cycles, reduced modulo one in binary64: phi0 of the
// first subcarrier (gain argument folded in), phiB per row block of B subcarriers and phi1
// per subcarrier (both kept in binary64, since a lane multiplies them by its row / column
// index 0..15), and p16B, p16_1 their 16-fold multiples (the step between 16-row tiles).
struct RecM {
  float amp, phi0, p16B, p16_1;
  double phiB, phi1;
};
// The same 32 bytes as four 64-bit words (amp | phi0, p16B | p16_1, phiB, phi1).
struct RecW { uint64_t w[4]; };
static_assert(sizeof(RecM) == sizeof(RecW), "RecM is four 64-bit words");
struct RecD { double L, gr, gi, zr, zi; };              // binary64: 40 B
struct RecN { float L, gr, gi, zr, zi, pad; };          // naive binary32: 24 B

}  // namespace drt

#endif  // DRT_RECORDS_H
