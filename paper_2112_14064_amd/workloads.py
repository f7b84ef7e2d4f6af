"""Seeded synthetic workloads for the damped-wave QEP on the unit square.

This module only *describes* problem instances and draws their random inputs
(per-element damping fields, batched-instance parameters, Krylov start blocks).
It contains none of the method's arithmetic, so both the HIP path and the
CPU oracle used by the tests can draw identical inputs from it.

The paper's efficiency study (Sec. 6.3) sweeps meshes of 2^s x 2^s elements,
degrees p = 3..6 and 16 x 16-element macroelements; the configurations below
are scalar H^1 stand-ins of that study (the paper measures no dataset: its
workloads are PDE discretisations, Sec. 6.3).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Problem:
    """One QEP instance: mesh, B-spline space, damping, shift and solve sizes.

    p            B-spline degree (Sec. 3.1)
    ne           elements per direction on (0,1)^2
    hyper_every  rIGA: C^0 hyperplanes every `hyper_every` elements (Sec. 3.3);
                 0 means maximum-continuity IGA (Sec. 3.2)
    alpha, beta  Rayleigh part of the damping, C = alpha*M + beta*K (+ elementwise)
    c_elem       optional per-element viscous coefficients, shape (ne, ne) indexed
                 [ey, ex]; adds sum_e c_e M_e to C
    sigma        real positive shift of the spectral transformation (Sec. 4.1.1)
    nev, m       requested eigenpairs and Krylov subspace size (Alg. 2)
    """

    p: int
    ne: int
    hyper_every: int
    alpha: float = 0.0
    beta: float = 0.0
    c_elem: Optional[np.ndarray] = None
    sigma: float = 1.0
    nev: int = 10
    m: int = 20
    name: str = ""
    extra: dict = field(default_factory=dict)


def lognormal_field(ne: int, seed: int, mean: float = -3.0, sd: float = 0.5) -> np.ndarray:
    """Per-element damping c_e ~ lognormal(mean, sd), shape (ne, ne) = [ey, ex]."""
    rng = np.random.default_rng(seed)
    return rng.lognormal(mean, sd, size=(ne, ne))


def start_block(ndof: int, block: int, seed: int) -> np.ndarray:
    """Gaussian start block for the Krylov iteration, shape (block, 2*ndof).

    A random start is required: a constant vector lies in the subspace that
    is symmetric under the x<->y reflection of the square and never sees the
    antisymmetric eigenmodes.
    """
    rng = np.random.default_rng(seed)
    return rng.standard_normal((block, 2 * ndof))


def random_rhs(ndof: int, nrhs: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nrhs, ndof))


# --- the five configurations -------------------------------------------------

def cfg_small() -> Problem:
    """p=2 on 16x16, C^0 hyperplanes every 4 elements, Rayleigh 0.1 M + 0.01 K,
    10 eigenvalues nearest sigma=1 (361 dofs)."""
    return Problem(p=2, ne=16, hyper_every=4, alpha=0.1, beta=0.01, sigma=1.0,
                   nev=10, m=20, name="p2_16x16_s4")


def cfg_riga_vs_iga(hyper_every: int = 16) -> Problem:
    """p=3 on 256x256, rIGA (C^0 every 16 elements) or IGA (hyper_every=0),
    Rayleigh 0.05 M + 0.005 K, 40 eigenpairs nearest sigma=2, subspace 80."""
    tag = f"s{hyper_every}" if hyper_every else "iga"
    return Problem(p=3, ne=256, hyper_every=hyper_every, alpha=0.05, beta=0.005,
                   sigma=2.0, nev=40, m=80, name=f"p3_256x256_{tag}")


def cfg_undamped(hyper_every: int = 16) -> Problem:
    """The undamped case (C = 0: K u = mu M u) on the headline mesh, p=3 on
    256x256, rIGA (C^0 every 16 elements) or IGA (hyper_every=0): every
    eigenvalue in [0, 1500) (108 with multiplicity) by spectrum slicing
    with at most 40 eigenvalues per slice."""
    tag = f"s{hyper_every}" if hyper_every else "iga"
    return Problem(p=3, ne=256, hyper_every=hyper_every, name=f"p3_256x256_{tag}_undamped",
                   extra={"interval": (0.0, 1500.0), "max_slice": 40})


def cfg_gyro(hyper_every: int = 16) -> Problem:
    """The headline mesh with a gyroscopic damping: p=3 on 256x256, rIGA (C^0
    every 16 elements) or IGA (hyper_every=0), C = 0.05 M + 0.005 K + G with
    the skew form of g = (0.5, 0), the 40 eigenpairs nearest sigma=2 with
    subspace 80."""
    tag = f"s{hyper_every}" if hyper_every else "iga"
    return Problem(p=3, ne=256, hyper_every=hyper_every, alpha=0.05, beta=0.005, sigma=2.0, nev=40, m=80,
                   name=f"p3_256x256_{tag}_gyro", extra={"gyro": (0.5, 0.0)})


def cfg_precision() -> Problem:
    """p=4 on 1024x1024, C^0 every 32 elements, c_e ~ lognormal(-3,0.5) seed 0,
    20 eigenpairs near sigma=5."""
    return Problem(p=4, ne=1024, hyper_every=32, c_elem=lognormal_field(1024, 0),
                   sigma=5.0, nev=20, m=40, name="p4_1024x1024_s32")


def cfg_batch(n: int = 256, seed: int = 1) -> list:
    """n independent instances: ne in {32,48,64,96,128}, p in {2,3,4}, s=8,
    alpha~U[0,0.2], beta~U[0,0.02], sigma~U[0.5,4]; 8 eigenpairs, subspace 20.
    Draw order: ne index, p, alpha, beta, sigma (each vectorised over n)."""
    rng = np.random.default_rng(seed)
    nes = np.array([32, 48, 64, 96, 128])
    ne_i = rng.integers(0, len(nes), size=n)
    ps = rng.integers(2, 5, size=n)
    al = rng.uniform(0.0, 0.2, size=n)
    be = rng.uniform(0.0, 0.02, size=n)
    sg = rng.uniform(0.5, 4.0, size=n)
    return [Problem(p=int(ps[k]), ne=int(nes[ne_i[k]]), hyper_every=8, alpha=float(al[k]),
                    beta=float(be[k]), sigma=float(sg[k]), nev=8, m=20, name=f"batch{k}")
            for k in range(n)]


def cfg_adjoint() -> Problem:
    """p=3 on 512x512, C^0 every 16 elements, c_e ~ lognormal(-3,0.5) seed 2,
    L = sum Re(lambda_k) over 20 eigenvalues nearest sigma=2."""
    return Problem(p=3, ne=512, hyper_every=16, c_elem=lognormal_field(512, 2),
                   sigma=2.0, nev=20, m=40, name="p3_512x512_s16")


def fd_elements(ne: int, count: int = 32, seed: int = 2) -> np.ndarray:
    """Elements (flat index ey*ne+ex) probed by finite differences of the adjoint."""
    rng = np.random.default_rng(seed)
    rng.lognormal(-3.0, 0.5, size=(ne, ne))  # same stream position as the field draw
    return rng.choice(ne * ne, size=count, replace=False)


def cfg_hcurl(hyper_every: int = 16) -> Problem:
    """The curl-conforming space S^{2,3} x S^{3,2} (p=3) on 256x256 with the
    perfect-conductor condition, rIGA (C^1/C^0 hyperplanes every 16 elements,
    148,512 dofs) or IGA (hyper_every=0, 132,612 dofs): the conductive form
    C = 0.05 M + 0.005 K factored at sigma=2 and solved with two right-hand
    sides, and the non-conductive (Maxwell) form K u = mu M u with every
    eigenvalue in [1, 150) by spectrum slicing, at most 40 per slice."""
    tag = f"s{hyper_every}" if hyper_every else "iga"
    return Problem(p=3, ne=256, hyper_every=hyper_every, alpha=0.05, beta=0.005, sigma=2.0,
                   name=f"p3_256x256_{tag}_hcurl", extra={"space": 1, "interval": (1.0, 150.0), "max_slice": 40})


def cfg_em_qep(hyper_every: int = 16) -> Problem:
    """The conductive electromagnetic QEP on the curl-conforming space S^{2,3} x
    S^{3,2} (p=3) on 256x256 with the perfect conductor, rIGA (C^1/C^0
    hyperplanes every 16 elements) or IGA (hyper_every=0): C = 0.05 M +
    0.005 K, complex target sigma = 7i, the 38 pairs of largest |psi| (a gap
    of the spectrum: no conjugate cluster is split), subspace 80."""
    tag = f"s{hyper_every}" if hyper_every else "iga"
    return Problem(p=3, ne=256, hyper_every=hyper_every, alpha=0.05, beta=0.005, sigma=7.0, nev=38, m=80,
                   name=f"p3_256x256_{tag}_em_qep", extra={"space": 1, "sigma_c": 7.0j})


def cfg_vibroacoustic(hyper_every: int = 16) -> Problem:
    """The vibroacoustic QEP of an acoustic cavity (the divergence-conforming
    space S^{3,2} x S^{2,3}, p=3, on 256x256): rigid walls except an absorbing
    top wall with coefficients alpha = 0.5, beta = 0.8 (rho = c = 1), rIGA
    (C^1/C^0 hyperplanes every 16 elements) or IGA (hyper_every=0); the 40
    pairs of largest |psi| at the complex target 0.5 + 7i, subspace 80."""
    tag = f"s{hyper_every}" if hyper_every else "iga"
    return Problem(p=3, ne=256, hyper_every=hyper_every, alpha=0.5, beta=0.8, sigma=0.5, nev=40, m=80,
                   name=f"p3_256x256_{tag}_vibroacoustic",
                   extra={"space": 3, "walls": 8, "sigma_c": 0.5 + 7.0j})
