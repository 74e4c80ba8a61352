"""Seeded geometry and raw-basis generators for the synthetic workloads.

Element types carry even-tempered shells.  Where several shells of the same
angular momentum sit on one atom, the j-th of them takes the next three rungs
of the exponent ladder (k = 3j, 3j+1, 3j+2): read literally, two shells with
identical exponents would make the overlap matrix singular.
"""

import math

import numpy as np


def _ladder(base, ratio, k0, n=3):
    return [base * ratio ** (k0 + k) for k in range(n)]


# element type -> (Z, [(l, exponents, raw coefficients), ...])
ELEMENTS = {
    # H of the linear chain: one s shell, exponents 0.15 * 4^k, equal coefficients
    "Hc": (1.0, [(0, _ladder(0.15, 4.0, 0), [1.0, 1.0, 1.0])]),
    # O of the water-like molecules: s, s, p (0.2 * 3^k) and one d (0.8)
    "O": (8.0, [(0, _ladder(0.2, 3.0, 0), [1.0, 1.0, 1.0]),
                (0, _ladder(0.2, 3.0, 3), [1.0, 1.0, 1.0]),
                (1, _ladder(0.2, 3.0, 0), [1.0, 1.0, 1.0]),
                (2, [0.8], [1.0])]),
    # H of the water-like molecules: s, s, p (0.1 * 3^k)
    "Hw": (1.0, [(0, _ladder(0.1, 3.0, 0), [1.0, 1.0, 1.0]),
                 (0, _ladder(0.1, 3.0, 3), [1.0, 1.0, 1.0]),
                 (1, _ladder(0.1, 3.0, 0), [1.0, 1.0, 1.0])]),
    # C-like atom of the random-walk molecules: s, s, p, p (0.15 * 3^k)
    "C": (6.0, [(0, _ladder(0.15, 3.0, 0), [1.0, 1.0, 1.0]),
                (0, _ladder(0.15, 3.0, 3), [1.0, 1.0, 1.0]),
                (1, _ladder(0.15, 3.0, 0), [1.0, 1.0, 1.0]),
                (1, _ladder(0.15, 3.0, 3), [1.0, 1.0, 1.0])]),
    # H-like atom of the random-walk molecules: s, p (0.1 * 3^k)
    "Hr": (1.0, [(0, _ladder(0.1, 3.0, 0), [1.0, 1.0, 1.0]),
                 (1, _ladder(0.1, 3.0, 0), [1.0, 1.0, 1.0])]),
}

_NCART = (1, 3, 6)


def nbf_of(basis):
    return int(sum(_NCART[l] for l in basis["shell_l"]))


def assemble(types, xyz, name="molecule", charge=0):
    """Build the raw basis dict for atoms of the given element types."""
    xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1, 3))
    assert len(types) == xyz.shape[0]
    Z, sa, sl, sn, sp, ex, co = [], [], [], [], [], [], []
    for a, t in enumerate(types):
        z, shells = ELEMENTS[t]
        Z.append(z)
        for (l, e, c) in shells:
            sa.append(a)
            sl.append(l)
            sn.append(len(e))
            sp.append(len(ex))
            ex.extend(e)
            co.extend(c)
    nelec = int(round(sum(Z))) - charge
    return {
        "xyz": xyz,
        "Z": np.asarray(Z, dtype=np.float64),
        "shell_atom": np.asarray(sa, dtype=np.int32),
        "shell_l": np.asarray(sl, dtype=np.int32),
        "shell_nprim": np.asarray(sn, dtype=np.int32),
        "shell_prim0": np.asarray(sp, dtype=np.int32),
        "exps": np.asarray(ex, dtype=np.float64),
        "coefs": np.asarray(co, dtype=np.float64),
        "nelec": nelec,
        "name": name,
        "types": list(types),
    }


def h_chain(natom=8, spacing=1.4):
    """Linear H chain along z, atom i at z = spacing * i."""
    xyz = np.zeros((natom, 3))
    xyz[:, 2] = spacing * np.arange(natom)
    return assemble(["Hc"] * natom, xyz, name=f"H{natom}-chain")


def cube_edge(nmol):
    """Cube edge for n water-like molecules: 14 bohr at n=10, 26 bohr at n=64."""
    return 14.0 * (nmol / 10.0) ** (1.0 / 3.0)


def _random_rotation(rng):
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def water_cluster(nmol, seed, edge=None, min_oo=5.0, r_oh=1.81, angle_deg=104.5):
    """n water-like molecules: O uniform in a cube with an O-O rejection
    distance; each molecule rigid (O-H 1.81 bohr, HOH 104.5 deg) under a
    uniform random orientation."""
    rng = np.random.default_rng(seed)
    L = cube_edge(nmol) if edge is None else edge
    oxy = []
    tries = 0
    while len(oxy) < nmol:
        tries += 1
        if tries > 1_000_000:
            raise RuntimeError("water placement failed; cube too small")
        o = rng.uniform(0.0, L, size=3)
        if all(np.linalg.norm(o - p) >= min_oo for p in oxy):
            oxy.append(o)
    th = math.radians(angle_deg)
    h1 = np.array([r_oh, 0.0, 0.0])
    h2 = np.array([r_oh * math.cos(th), r_oh * math.sin(th), 0.0])
    types, xyz = [], []
    for o in oxy:
        R = _random_rotation(rng)
        types += ["O", "Hw", "Hw"]
        xyz += [o, o + R @ h1, o + R @ h2]
    return assemble(types, np.array(xyz), name=f"(H2O){nmol}-seed{seed}")


def ch_molecule(seed, nmin=2, nmax=24, bond=(2.0, 2.9), min_dist=1.8):
    """Random-walk C/H molecule: atom count uniform in [nmin, nmax], types
    i.i.d. with P(C) = 1/2, each atom placed from the previous one at a
    uniform bond length in a uniform direction, redrawn while any atom is
    closer than min_dist.  An odd electron count flips the last atom's type."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(nmin, nmax + 1))
    types = ["C" if rng.random() < 0.5 else "Hr" for _ in range(n)]
    pos = [np.zeros(3)]
    for k in range(1, n):
        for _ in range(10_000):
            d = rng.standard_normal(3)
            d /= np.linalg.norm(d)
            cand = pos[-1] + rng.uniform(*bond) * d
            if all(np.linalg.norm(cand - p) >= min_dist for p in pos):
                break
        else:
            raise RuntimeError("random walk got stuck")
        pos.append(cand)
    ztot = sum(ELEMENTS[t][0] for t in types)
    if int(round(ztot)) % 2 == 1:
        types[-1] = "Hr" if types[-1] == "C" else "C"
    return assemble(types, np.array(pos), name=f"CH{n}-seed{seed}")


def batch_molecules(count=1024, seed0=4_000_000, **kw):
    return [ch_molecule(seed0 + i, **kw) for i in range(count)]


# The synthetic workloads, with the screening / precision settings that go with them.
WORKLOADS = {
    "h8_chain": dict(kind="h_chain", natom=8, spacing=1.4, tau=0.0, tau_fp32=0.0,
                     conv_rms_dD=1e-10, conv_dE=0.0),
    "water10": dict(kind="water", nmol=10, seed=2, tau=1e-12, tau_fp32=0.0,
                    conv_rms_dD=1e-8, conv_dE=1e-10),
    "water64": dict(kind="water", nmol=64, seed=3, tau=1e-11, tau_fp32=1e-5,
                    conv_rms_dD=1e-8, conv_dE=1e-10),
    # 1024 random-walk C/H molecules of 2-24 atoms, run as one batch
    "ch1024": dict(kind="batch", count=1024, seed0=4_000_000, tau=1e-11, tau_fp32=1e-5,
                   conv_rms_dD=1e-8, conv_dE=1e-10),
}


def workload(name):
    """(basis, settings) for one of the named workloads."""
    w = dict(WORKLOADS[name])
    kind = w.pop("kind")
    if kind == "h_chain":
        b = h_chain(w.pop("natom"), w.pop("spacing"))
    elif kind == "water":
        b = water_cluster(w.pop("nmol"), w.pop("seed"))
    elif kind == "batch":
        b = batch_molecules(w.pop("count"), w.pop("seed0"))
    else:
        raise KeyError(kind)
    return b, w
