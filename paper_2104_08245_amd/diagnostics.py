"""Global checks of an assembled NOLSM density matrix (host side, scipy).

For D in block-CSR on the merged pattern and the overlap S (Sec. III-B.2,
write-back into D; D = (I - sign(S^-1 K - mu I)) S^-1 / 2 per submatrix):

  idempotency  ||D S D - D||_F / ||D||_F. The exact density matrix satisfies
               D S D = D; the submatrix truncation leaves a floor even when
               every submatrix is solved exactly, so a mixed-precision D is
               read against the FP64 D of the same method.
  asymmetry    ||D - D^T||_F / ||D||_F (the column write-back does not
               symmetrise D).
  trace        Tr(D S) per molecule (occupied orbitals per molecule).

With `probes` > 0, ||D S D - D||_F is estimated from Gaussian probe vectors:
E ||M z||^2 = ||M||_F^2 for z with independent zero-mean unit-variance
entries (Hutchinson's estimator), so sqrt(mean_k ||M z_k||^2) estimates
||M||_F with a relative standard error near 1 / sqrt(2 k). That avoids
forming D S D, whose pattern reaches three cutoff radii.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def block_csr(nb, bs, row_ptr, col_idx, blocks):
    """scipy CSR matrix of a square block-CSR matrix with bs x bs blocks."""
    m = sp.bsr_matrix((np.asarray(blocks, np.float64).reshape(-1, bs, bs), np.asarray(col_idx),
                       np.asarray(row_ptr)), shape=(nb * bs, nb * bs))
    return m.tocsr()


def density_checks(D, S, nmol, probes=0, seed=0):
    """dict(idempotency, asymmetry, trace_DS_per_molecule) of CSR matrices
    D and S; exact products when probes == 0, else the probe estimate."""
    nrm = spla.norm(D)
    if probes <= 0:
        idem = spla.norm(D @ S @ D - D) / nrm
    else:
        rng = np.random.default_rng(seed)
        Z = rng.standard_normal((D.shape[0], probes))
        DZ = D @ Z
        MZ = D @ (S @ DZ) - DZ
        idem = np.sqrt(np.square(MZ).sum() / probes) / nrm
    asym = spla.norm(D - D.T) / nrm
    tr = D.multiply(S.T).sum()
    return {"idempotency": float(idem), "asymmetry": float(asym), "trace_DS_per_molecule": float(tr / nmol)}
