"""Plain FP64 CPU oracle for the ETDM energy+gradient path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP library
(it imports only NumPy/SciPy and the seeded input generators in ``workloads``).

Modules
-------
etdm   : the definition path (eigendecomposition of iA, Eq. ed; the gradient of
         Eq. gradients through the eigenbasis of iA) and a structured
         occupied-virtual path (Hutter's parametrization, Eq. uinv, with the
         exact gradient derived from Eq. gradients).
lbfgs  : L-BFGS with the paper's preconditioner (Eq. prec_3 and Eq. betaij)
         and inexact line search (strong Wolfe, approximate Wolfe and energy
         conditions of Sec. 3.2).
scf    : a damped Roothaan SCF loop used only as an independent pin for the
         location of the energy minimum.

Parity status: every public function is pinned by tests under ``tests/``
(marked ``not gpu``); none is "parity unpinned".
"""
