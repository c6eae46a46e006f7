"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  This module holds random draws and problem shapes only; none of the
method's arithmetic lives here.

Right-hand sides are sums of Fourier modes
    f(x) = sum_q a_q prod_d sin(2 pi k_qd x_d / l_d + phi_qd)
whose parameters are drawn here (per mode, in this order: the three
wavenumbers in 1..kmax, the three phases in [0, 2 pi), the amplitude from a
standard normal).  Evaluating the load at the nodes and forming the discrete
right-hand side is done separately by each consumer.
"""

import dataclasses
import math

import numpy as np


def fourier_modes(seed, kmax, nmodes=20):
    """(k[nmodes, 3] int32, phi[nmodes, 3] float64, amp[nmodes] float64)."""
    rng = np.random.default_rng(seed)
    k = np.empty((nmodes, 3), dtype=np.int32)
    phi = np.empty((nmodes, 3))
    amp = np.empty(nmodes)
    for q in range(nmodes):
        k[q] = rng.integers(1, kmax + 1, 3)
        phi[q] = rng.uniform(0.0, 2.0 * math.pi, 3)
        amp[q] = rng.standard_normal()
    return k, phi, amp


def uniform_vector(seed, size, lo=-1.0, hi=1.0):
    """Seeded U[lo, hi] vector (random start values, random operands)."""
    return np.random.default_rng(seed).uniform(lo, hi, size)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    ne: tuple
    length: tuple
    P: int
    overlap: str          # 'min' | 'rel' | 'max'
    omega: float
    kmax: int
    solver: str           # 'mg' | 'fcg'
    growth: int = 1       # smoothing growth per coarser level (3 = variable V-cycle)

    @property
    def ndof(self):
        return self.ne[0] * self.ne[1] * self.ne[2] * (self.P + 1) ** 3


# The paper's isotropic study uses (128/P)^3 elements; the 16^3, P=8 case is
# its P=8 mesh.  The anisotropic case is the paper's 8^3, P=16 mesh with a
# 16:1:1 element aspect ratio and the "max" overlap of its Table 2.
WORKLOADS = {
    "cube4_p4_min": Workload("cube4_p4_min", (4, 4, 4), (1.0, 1.0, 1.0), 4, "min", 0.08, 3, "mg"),
    "cube16_p8_rel": Workload("cube16_p8_rel", (16, 16, 16), (1.0, 1.0, 1.0), 8, "rel", 0.08, 8, "mg"),
    "aniso16_p16_max": Workload("aniso16_p16_max", (8, 8, 8), (16.0, 1.0, 1.0), 16, "max", 0.08, 3, "fcg"),
    "cube32_p7_rel": Workload("cube32_p7_rel", (32, 32, 32), (1.0, 1.0, 1.0), 7, "rel", 0.08, 8, "fcg"),
    # one GPU's share of a large job: 64^3 elements, 134,217,728 unknowns
    "cube64_p7_rel": Workload("cube64_p7_rel", (64, 64, 64), (1.0, 1.0, 1.0), 7, "rel", 0.08, 8, "fcg"),
}


def serving_stream_same_order(seed, nreq, qps, P=8, ne_range=(4, 7)):
    """Poisson arrivals of small solves of one order on isotropic meshes
    (edge element count uniform in ne_range, independently per direction,
    unit element aspect ratio): every request has the same preconditioner
    signature, so ready requests can share their V-cycle launches."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(nreq):
        t += rng.exponential(1.0 / qps)
        ne = tuple(int(v) for v in rng.integers(ne_range[0], ne_range[1] + 1, size=3))
        out.append({"id": i, "t_arrival": t, "ne": ne, "P": int(P),
                    "length": tuple(float(v) for v in ne), "rhs_seed": int(rng.integers(0, 2 ** 31))})
    return out


def serving_stream(seed, nreq, qps):
    """Poisson arrivals of heterogeneous solves: per request the edge element
    count (uniform 4..24, same in every direction), the order from
    {2, 4, 8, 16, 32}, the aspect ratio 1..8 with l = (AR, 1, 1), and the
    right-hand-side seed.  Returns a list of dicts sorted by arrival time."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(nreq):
        t += rng.exponential(1.0 / qps)
        ne = int(rng.integers(4, 25))
        P = int(rng.choice([2, 4, 8, 16, 32]))
        ar = int(rng.integers(1, 9))
        out.append({"id": i, "t_arrival": t, "ne": (ne, ne, ne), "P": P,
                    "length": (float(ar), 1.0, 1.0), "rhs_seed": int(rng.integers(0, 2 ** 31))})
    return out
