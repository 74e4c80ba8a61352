"""Small builders for test molecules (raw basis dicts in the synth format)."""

import numpy as np

import synth


def custom_basis(atoms, nelec=None, name="custom"):
    """atoms: list of (xyz, Z, [(l, [exps], [coefs]), ...])."""
    xyz, Z, sa, sl, sn, sp, ex, co = [], [], [], [], [], [], [], []
    for a, (pos, z, shells) in enumerate(atoms):
        xyz.append(pos)
        Z.append(z)
        for (l, e, c) in shells:
            sa.append(a)
            sl.append(l)
            sn.append(len(e))
            sp.append(len(ex))
            ex.extend(e)
            co.extend(c)
    if nelec is None:
        nelec = int(round(sum(Z)))
    return {
        "xyz": np.asarray(xyz, dtype=np.float64).reshape(-1, 3),
        "Z": np.asarray(Z, dtype=np.float64),
        "shell_atom": np.asarray(sa, dtype=np.int32),
        "shell_l": np.asarray(sl, dtype=np.int32),
        "shell_nprim": np.asarray(sn, dtype=np.int32),
        "shell_prim0": np.asarray(sp, dtype=np.int32),
        "exps": np.asarray(ex, dtype=np.float64),
        "coefs": np.asarray(co, dtype=np.float64),
        "nelec": int(nelec),
        "name": name,
    }


def transformed(basis, R=None, shift=None):
    """Same molecule after a rigid rotation R and a shift."""
    b = dict(basis)
    x = np.array(basis["xyz"], dtype=np.float64)
    if R is not None:
        x = x @ np.asarray(R).T
    if shift is not None:
        x = x + np.asarray(shift)
    b["xyz"] = np.ascontiguousarray(x)
    return b


def random_rotation(rng):
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def water(nmol=1, seed=0):
    return synth.water_cluster(nmol, seed)


def spd_molecule():
    """Three atoms with s, p and d shells of mixed contraction, for ERI checks."""
    return custom_basis([
        ([0.0, 0.0, 0.0], 8.0, [(0, [5.0, 1.1], [0.4, 0.7]), (1, [1.3, 0.35], [0.5, 0.6]),
                                 (2, [0.8], [1.0])]),
        ([1.2, 0.4, -0.3], 1.0, [(0, [0.9, 0.2], [0.6, 0.5]), (1, [0.6], [1.0])]),
        ([-0.5, 1.1, 0.9], 1.0, [(2, [0.5, 1.7], [0.7, 0.3]), (0, [0.45], [1.0])]),
    ], nelec=10)
