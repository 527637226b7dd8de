"""Reference (oracle) POD of a snapshot set by the method of snapshots.

TEST INFRASTRUCTURE ONLY.  Only the tests and the benchmark's CPU-baseline
leg may import this module.  It shares no code with the HIP path.

What it computes (arXiv 1704.04139, Sec. 2.5 "Model order reduction and
reduced simulation"): the reduced spaces for the concentration and the
potential are spanned by the leading POD (principal component) modes of the
snapshot sets, which hold the solution at every time step and the
intermediate Newton stages.  The POD is taken by the method of snapshots
(Sirovich 1987, the reference the paper gives):

  1. correlation (Gram) matrix  K = S^T W S  of the m snapshots, W the
     diagonal weight of the inner product (identity: Euclidean);
  2. eigen-decomposition  K = V diag(lam) V^T, eigenvalues descending;
  3. singular values  sigma_i = sqrt(max(lam_i, 0));
  4. modes  u_i = S v_i / sigma_i  for the kept i.

Readings (the paper is silent on them): the inner product is Euclidean on
the voxel values unless a weight is given; a mode is kept while
sigma_i > rtol * sigma_1 (the experiment of Sec. 3.2 uses rtol = 1e-7), at most
k_max of them; the sign of each mode is fixed by making the entry of largest
magnitude of its coefficient vector v_i positive (first such entry on ties).

Pins (tests/test_pod_pins.py): the singular values equal those of an SVD
of W^(1/2) S; a snapshot set built from a prescribed orthonormal basis and
spectrum returns that spectrum and basis; the projection error obeys the
Eckart-Young identity; the modes are W-orthonormal; a single snapshot gives
its own normalised direction.
Precision: float64 throughout.
"""
import numpy as np


def gram(S, w=None):
    """Step 1: K = S^T W S (W = diag(w), identity when w is None)."""
    S = np.asarray(S, dtype=np.float64)
    if w is None:
        return S.T @ S
    return S.T @ (np.asarray(w, dtype=np.float64)[:, None] * S)


def pod(S, w=None, rtol=1e-7, k_max=None):
    """Method-of-snapshots POD of the columns of S (n x m).

    Returns (modes n x k, sigma (all m singular values, descending),
    V m x k coefficient vectors of the kept modes)."""
    S = np.asarray(S, dtype=np.float64)
    n, m = S.shape
    K = gram(S, w)
    lam, V = np.linalg.eigh(K)                 # step 2 (ascending from the library)
    order = np.argsort(lam)[::-1]
    lam, V = lam[order], V[:, order]
    sigma = np.sqrt(np.maximum(lam, 0.0))      # step 3
    if k_max is None:
        k_max = m
    keep = 0
    while keep < min(k_max, m) and sigma[keep] > rtol * sigma[0] and sigma[keep] > 0.0:
        keep += 1
    V = V[:, :keep].copy()
    for i in range(keep):                      # sign convention
        j = int(np.argmax(np.abs(V[:, i])))
        if V[j, i] < 0.0:
            V[:, i] = -V[:, i]
    modes = S @ (V / sigma[:keep])             # step 4
    return modes, sigma, V
