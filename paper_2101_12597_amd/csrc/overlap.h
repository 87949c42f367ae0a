// Non-orthogonal basis (Sec. 2: orbitals O with O^H S O = I): the Lowdin transform
// H0' = S^-1/2 H0 S^-1/2, C0' = S^1/2 C0 turns the problem into the orthonormal one
// (the site populations of the model become the Lowdin populations).  S^1/2 and
// S^-1/2 come from the coupled Newton-Schulz iteration on S / c, c >= the largest
// eigenvalue (a Gershgorin bound):
//   P = Z Y,  T = (3 I - P) / 2,  Y <- Y T,  Z <- T Z,   Y -> (S/c)^1/2, Z -> (S/c)^-1/2,
// whose products are grouped GEMMs launched by the caller.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace etdm {

// Per instance: M x M matrices, real (cplx = 0) or interleaved complex, row-major.
struct OvlInst {
  const double* S;  // overlap (read)
  double *Y, *Z;    // iterate of the current parity (Y, Z at start: S / c, I)
  double *P, *T;    // Z Y and (3 I - P) / 2
  double* c;        // the scale c (one double)
  int32_t M;
};

// c = largest row sum of |S_ij| per instance, then Y = S / c and Z = I
void launch_ovl_start(const OvlInst* d, const int* d_begin, int n_inst, int total, int cplx, hipStream_t s);
// T = (3 I - P) / 2 and resid[i] = max |I - P| of instance i (one workgroup per instance)
void launch_ovl_step(const OvlInst* d, int n_inst, int cplx, double* resid, hipStream_t s);
// Y <- sqrt(c) Y (= S^1/2), Z <- Z / sqrt(c) (= S^-1/2)
void launch_ovl_finish(const OvlInst* d, const int* d_begin, int n_inst, int total, int cplx, hipStream_t s);

}  // namespace etdm
