"""Seeded synthetic molecules and raw basis data.

This module is the only code shared by the oracle and the GPU path.  It makes
geometries, nuclear charges and *raw* basis data (shell centres, angular
momenta, exponents and unnormalised contraction coefficients) and nothing else:
no normalisation, no integrals, no part of the Hartree-Fock arithmetic.  Each
side normalises the primitives and contracted functions on its own.

A basis is a plain dict of numpy arrays:

    xyz          (natom, 3) float64, bohr
    Z            (natom,)   float64, nuclear charges
    shell_atom   (nshell,)  int32, atom index of each shell
    shell_l      (nshell,)  int32, 0 (s), 1 (p) or 2 (Cartesian d)
    shell_nprim  (nshell,)  int32
    shell_prim0  (nshell,)  int32, offset of the shell's primitives
    exps, coefs  (nprim_total,) float64, raw exponents and coefficients
    nelec        int, even (closed shell)
    name         str
"""

from .molecules import (  # noqa: F401
    ELEMENTS,
    assemble,
    h_chain,
    water_cluster,
    ch_molecule,
    batch_molecules,
    nbf_of,
    cube_edge,
    WORKLOADS,
    workload,
)
