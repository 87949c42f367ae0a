// Large symmetric eigensolver (block-cyclic Jacobi with matrix-core updates).
#pragma once

#include <algorithm>

#include "common.h"

namespace etdm {

struct EighLargeState {
  double scale;                  // ||A||_F
  unsigned long long sweep_off;  // bit pattern of the largest off-diagonal |a_ik| after the sweep
  int sweeps;
  int done;
  int finite;
};

struct EighLarge {
  const double* P;  // n x n input (its symmetric part is used)
  double* X;        // n x n eigenvectors (columns)
  double* w;        // n eigenvalues (unsorted)
  double* Aw;       // npad x npad work matrix
  double* Vw;       // npad x npad accumulated rotations
  double* Qb;       // (nb / 2) x 64 x 64 rotations of one round
  double* partial;  // reduction scratch (256 doubles)
  EighLargeState* st;
  int n, npad, nb;
};

// float64 elements of workspace for size n (Aw, Vw, Qb, partial); npad returned.
size_t eigh_large_workspace(int n, size_t* npad_out);
// Launch the whole solve on stream s.  With check_host the host reads the
// convergence flag after every sweep and stops launching early (not usable
// under graph capture); otherwise all max_sweeps sweeps are launched and the
// ones after convergence return immediately.
void launch_eigh_large(const EighLarge& e, int max_sweeps, int* status, hipStream_t s, bool check_host);

}  // namespace etdm
