"""Python binding of libfsim.so (the C ABI in include/fsim.h).

Argument marshalling only: torch provides device memory and the current
stream; every step of the Fock build and the SCF step runs in the library's
kernels.  There is no fallback: without a built libfsim.so, or without a
GPU, every entry point raises.
"""

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libfsim.so")
_lib = None

FSIM_FP64 = 0
FSIM_MIXED = 1
_PREC = {"fp64": FSIM_FP64, "mixed": FSIM_MIXED}
NCART = (1, 3, 6)


class FsimError(RuntimeError):
    pass


class _Basis(ctypes.Structure):
    _fields_ = [("natom", ctypes.c_int32), ("xyz", ctypes.c_void_p), ("Z", ctypes.c_void_p),
                ("nshell", ctypes.c_int32), ("shell_atom", ctypes.c_void_p),
                ("shell_l", ctypes.c_void_p), ("shell_nprim", ctypes.c_void_p),
                ("shell_prim0", ctypes.c_void_p), ("exps", ctypes.c_void_p),
                ("coefs", ctypes.c_void_p), ("nelec", ctypes.c_int32)]


class _Options(ctypes.Structure):
    _fields_ = [("tau_screen", ctypes.c_double), ("tau_fp32", ctypes.c_double),
                ("diis_m", ctypes.c_int32), ("conv_rms_dD", ctypes.c_double),
                ("conv_dE", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("spherical", ctypes.c_int32)]


class _ScreenStats(ctypes.Structure):
    _fields_ = [("shell_pairs", ctypes.c_int64), ("pairs_kept", ctypes.c_int64),
                ("quartets_total", ctypes.c_int64), ("quartets_kept", ctypes.c_int64),
                ("quartets_fp64", ctypes.c_int64), ("quartets_fp32", ctypes.c_int64),
                ("prim_quartets_kept", ctypes.c_int64), ("flops_fp64", ctypes.c_double),
                ("flops_mixed_fp64", ctypes.c_double), ("flops_mixed_fp32", ctypes.c_double),
                ("prim_pairs_total", ctypes.c_int64), ("prim_pairs_kept", ctypes.c_int64)]


class _ScfInfo(ctypes.Structure):
    _fields_ = [("E_total", ctypes.c_double), ("E_elec", ctypes.c_double),
                ("dE", ctypes.c_double), ("rms_dD", ctypes.c_double),
                ("comm_norm", ctypes.c_double), ("iter", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("diis_used", ctypes.c_int32),
                ("full_build", ctypes.c_int32), ("quartets", ctypes.c_int64)]


class _ClassProfile(ctypes.Structure):
    _fields_ = [("bra_class", ctypes.c_int32), ("ket_class", ctypes.c_int32),
                ("fp32", ctypes.c_int32), ("tiles", ctypes.c_int32),
                ("quartets", ctypes.c_int64), ("prim_quartets", ctypes.c_int64),
                ("flops", ctypes.c_double), ("ms", ctypes.c_double),
                ("flops_exec", ctypes.c_double)]


class _Tuning(ctypes.Structure):
    _fields_ = [("bra_class", ctypes.c_int32), ("ket_class", ctypes.c_int32),
                ("fp32", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("waves_per_block", ctypes.c_int32), ("kbra", ctypes.c_int32),
                ("kket", ctypes.c_int32), ("seg_tiles", ctypes.c_int32),
                ("ms", ctypes.c_double)]


PAIR_CLASS = ("ss", "ps", "pp", "ds", "dp", "dd", "sp*")   # "sp*": the persistent s/p launch
NVARIANT = 7


def _struct_dict(s):
    return {name: getattr(s, name) for name, _ in s._fields_ if name != "pad"}


def lib():
    """Load libfsim.so (after torch, so both use one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise FsimError(f"{LIBPATH} is not built; run `python -m paper_2510_24968_amd.build`")
    L = ctypes.CDLL(LIBPATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.fsim_last_error.restype = ctypes.c_char_p
    L.fsim_version.restype = ctypes.c_char_p
    sigs = {
        "fsim_ctx_create": [ctypes.POINTER(_Basis), ctypes.POINTER(_Options),
                            ctypes.POINTER(vp)],
        "fsim_ctx_destroy": [vp],
        "fsim_nbf": [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "fsim_nuclear_repulsion": [vp, ctypes.POINTER(dbl)],
        "fsim_one_electron": [vp, vp, vp, vp, vp],
        "fsim_schwarz_screen": [vp, dbl, dbl, vp, ctypes.POINTER(_ScreenStats)],
        "fsim_fock_build": [vp, vp, vp, vp, vp, ctypes.POINTER(dbl), ctypes.c_int, vp],
        "fsim_fock_build_noalloc": [vp, vp, vp, vp, vp, ctypes.POINTER(dbl), ctypes.c_int, vp],
        "fsim_fock_build_delta": [vp, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(dbl), dbl,
                                  ctypes.POINTER(i64), ctypes.c_int, vp],
        "fsim_set_incremental": [vp, i32, dbl],
        "fsim_store_eris": [vp, i32, ctypes.POINTER(i64)],
        "fsim_core_guess": [vp, vp, vp],
        "fsim_scf_step": [vp, vp, ctypes.POINTER(_ScfInfo), ctypes.c_int, vp],
        "fsim_scf_reset": [vp],
        "fsim_eri_quartets": [vp, i64, vp, vp, vp, ctypes.c_int, vp],
        "fsim_set_profiling": [vp, i32],
        "fsim_batch_create": [vp, i32, ctypes.POINTER(_Options), ctypes.POINTER(vp)],
        "fsim_batch_layout": [vp, ctypes.POINTER(i32), vp, vp, vp, ctypes.POINTER(i64)],
        "fsim_batch_energies": [vp, vp],
        "fsim_batch_scf_info": [vp, vp],
        "fsim_set_graph": [vp, i32],
        "fsim_set_xcd_private": [vp, i32],
        "fsim_set_persistent": [vp, i32],
        "fsim_set_prim_screen": [vp, dbl],
        "fsim_set_krow_lds": [vp, i32],
        "fsim_set_tuning": [vp, vp, i32],
        "fsim_get_tuning": [vp, vp, i32, ctypes.POINTER(i32)],
        "fsim_autotune": [vp, vp, ctypes.c_int, vp],
        "fsim_get_class_profile": [vp, vp, i32, ctypes.POINTER(i32)],
    }
    for name, args in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    _lib = L
    return L


def _check(st):
    if st != 0:
        raise FsimError(f"fsim error {st}: {lib().fsim_last_error().decode()}")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def basis_struct(basis):
    """ctypes view of a synth-format basis dict (arrays kept alive by the caller)."""
    keep = [np.ascontiguousarray(basis["xyz"], dtype=np.float64).ravel(),
            np.ascontiguousarray(basis["Z"], dtype=np.float64),
            np.ascontiguousarray(basis["shell_atom"], dtype=np.int32),
            np.ascontiguousarray(basis["shell_l"], dtype=np.int32),
            np.ascontiguousarray(basis["shell_nprim"], dtype=np.int32),
            np.ascontiguousarray(basis["shell_prim0"], dtype=np.int32),
            np.ascontiguousarray(basis["exps"], dtype=np.float64),
            np.ascontiguousarray(basis["coefs"], dtype=np.float64)]
    b = _Basis(len(keep[1]), keep[0].ctypes.data, keep[1].ctypes.data, len(keep[2]),
               keep[2].ctypes.data, keep[3].ctypes.data, keep[4].ctypes.data,
               keep[5].ctypes.data, keep[6].ctypes.data, keep[7].ctypes.data,
               int(basis["nelec"]))
    return b, keep


class Context:
    """One molecule on the current GPU."""

    def __init__(self, basis, tau=0.0, tau_fp32=0.0, diis_m=8, conv_rms_dD=1e-8, conv_dE=1e-10,
                 max_iter=100, device="cuda", spherical=False):
        L = lib()
        if not torch.cuda.is_available():
            raise FsimError("no GPU: libfsim runs on an MI355X only")
        self.device = torch.device(device)
        b, keep = basis_struct(basis)
        self.opt = _Options(float(tau), float(tau_fp32), int(diis_m), float(conv_rms_dD),
                            float(conv_dE), int(max_iter), 1 if spherical else 0)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(L.fsim_ctx_create(ctypes.byref(b), ctypes.byref(self.opt), ctypes.byref(h)))
        self.h = h
        n, ns = ctypes.c_int32(), ctypes.c_int32()
        _check(L.fsim_nbf(self.h, ctypes.byref(n), ctypes.byref(ns)))
        self.nbf, self.nshell = n.value, ns.value
        e = ctypes.c_double()
        _check(L.fsim_nuclear_repulsion(self.h, ctypes.byref(e)))
        self.enuc = e.value
        self.nelec = int(basis["nelec"])
        self.tau, self.tau_fp32 = float(tau), float(tau_fp32)
        self.tau_prim = 0.0
        self.shell_l = np.asarray(basis["shell_l"], dtype=np.int32)
        self.packed = self.nbf * self.nbf
        self.screen_stats = None

    def close(self):
        if getattr(self, "h", None):
            lib().fsim_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _mat(self):
        return torch.empty((self.nbf, self.nbf), dtype=torch.float64, device=self.device)

    def one_electron(self):
        S, H, X = self._mat(), self._mat(), self._mat()
        _check(lib().fsim_one_electron(self.h, _ptr(S), _ptr(H), _ptr(X), _stream()))
        return S, H, X

    def schwarz_screen(self, tau=None, tau_fp32=None, want_q=True):
        tau = self.tau if tau is None else float(tau)
        tau_fp32 = self.tau_fp32 if tau_fp32 is None else float(tau_fp32)
        Q = torch.empty((self.nshell, self.nshell), dtype=torch.float64, device=self.device) \
            if want_q else None
        st = _ScreenStats()
        torch.cuda.current_stream().synchronize()
        _check(lib().fsim_schwarz_screen(self.h, tau, tau_fp32, _ptr(Q), ctypes.byref(st)))
        self.screen_stats = _struct_dict(st)
        return Q, self.screen_stats

    def fock_build(self, D, precision="fp64", want_jk=False, energy=True, F=None):
        assert D.dtype == torch.float64 and D.is_contiguous() and D.numel() == self.packed
        F = self._mat() if F is None else F
        J = self._mat() if want_jk else None
        K = self._mat() if want_jk else None
        e = ctypes.c_double()
        _check(lib().fsim_fock_build(self.h, _ptr(D), _ptr(F), _ptr(J), _ptr(K),
                                     ctypes.byref(e) if energy else None, _PREC[precision],
                                     _stream()))
        return {"F": F, "J": J, "K": K, "E_elec": e.value if energy else None}

    def fock_build_noalloc(self, D, F, J=None, K=None, precision="fp64", energy=True):
        """fsim_fock_build_noalloc into caller-allocated F (and J, K): the
        call allocates no device memory."""
        assert D.dtype == torch.float64 and D.is_contiguous() and D.numel() == self.packed
        e = ctypes.c_double()
        _check(lib().fsim_fock_build_noalloc(self.h, _ptr(D), _ptr(F), _ptr(J), _ptr(K),
                                             ctypes.byref(e) if energy else None,
                                             _PREC[precision], _stream()))
        return e.value if energy else None

    def fock_build_delta(self, D, D_ref, J_ref, K_ref, precision="fp64", in_place=False,
                         tau_delta=0.0):
        """J = J_ref + J[D - D_ref], K = K_ref + K[D - D_ref] over the
        quartets whose density-weighted bound reaches tau_delta (0: the
        screen's tau), F = H + J - K/2 (fsim_fock_build_delta).  in_place
        updates J_ref and K_ref."""
        for t in (D, D_ref, J_ref, K_ref):
            assert t.dtype == torch.float64 and t.is_contiguous() and t.numel() == self.packed
        F = self._mat()
        J = J_ref if in_place else self._mat()
        K = K_ref if in_place else self._mat()
        e = ctypes.c_double()
        nq = ctypes.c_int64()
        _check(lib().fsim_fock_build_delta(self.h, _ptr(D), _ptr(D_ref), _ptr(J_ref), _ptr(K_ref),
                                           _ptr(F), _ptr(J), _ptr(K), ctypes.byref(e),
                                           float(tau_delta), ctypes.byref(nq), _PREC[precision],
                                           _stream()))
        return {"F": F, "J": J, "K": K, "E_elec": e.value, "quartets": nq.value}

    def store_eris(self, enable=True):
        """Conventional mode: compute every kept quartet once and digest the
        stored blocks in later builds (fsim_store_eris); returns the bytes."""
        nb = ctypes.c_int64()
        _check(lib().fsim_store_eris(self.h, 1 if enable else 0, ctypes.byref(nb)))
        return nb.value

    def set_incremental(self, rebuild_every, tau_delta=0.0):
        """SCF steps with incremental Fock builds (density-weighted threshold
        tau_delta, 0: the screen's tau) and a full build every rebuild_every
        steps (0: always full)."""
        _check(lib().fsim_set_incremental(self.h, int(rebuild_every), float(tau_delta)))

    def core_guess(self):
        D = self._mat()
        _check(lib().fsim_core_guess(self.h, _ptr(D), _stream()))
        return D

    def scf_reset(self):
        _check(lib().fsim_scf_reset(self.h))

    def scf_step(self, D, precision="fp64"):
        info = _ScfInfo()
        _check(lib().fsim_scf_step(self.h, _ptr(D), ctypes.byref(info), _PREC[precision],
                                   _stream()))
        return _struct_dict(info)

    def set_xcd_private(self, enable=True):
        """Per-XCD private J'/K' accumulators (default on) or one shared copy."""
        _check(lib().fsim_set_xcd_private(self.h, 1 if enable else 0))

    def set_graph(self, enable=True):
        """Replay Fock builds that ask for F only from a captured hipGraph
        (fsim_set_graph)."""
        _check(lib().fsim_set_graph(self.h, 1 if enable else 0))

    def set_krow_lds(self, enable=True):
        """K' rows of each bra accumulated in LDS over segments of its tiles
        (default) or every K' term added globally (fsim_set_krow_lds)."""
        _check(lib().fsim_set_krow_lds(self.h, 1 if enable else 0))

    def set_prim_screen(self, tau_prim):
        """Primitive-pair screening at tau_prim (0: off) for the next
        schwarz_screen (fsim_set_prim_screen); the current screen is
        invalidated."""
        _check(lib().fsim_set_prim_screen(self.h, float(tau_prim)))
        self.tau_prim = float(tau_prim)

    def set_persistent(self, enable=True):
        """s/p quartet classes in one persistent queue launch per precision
        part (fsim_set_persistent)."""
        _check(lib().fsim_set_persistent(self.h, 1 if enable else 0))

    def set_profiling(self, enable=True):
        _check(lib().fsim_set_profiling(self.h, 1 if enable else 0))

    def class_profile(self):
        """Per-launch records of the last profiled Fock build."""
        n = ctypes.c_int32()
        _check(lib().fsim_get_class_profile(self.h, None, 0, ctypes.byref(n)))
        arr = (_ClassProfile * max(1, n.value))()
        _check(lib().fsim_get_class_profile(self.h, arr, n.value, ctypes.byref(n)))
        out = []
        for k in range(n.value):
            d = _struct_dict(arr[k])
            d["cls"] = f"({PAIR_CLASS[d['bra_class']]}|{PAIR_CLASS[d['ket_class']]})"
            out.append(d)
        return out

    def get_tuning(self):
        """Launch settings of every (bra class, ket class, precision)."""
        n = ctypes.c_int32()
        arr = (_Tuning * 64)()
        _check(lib().fsim_get_tuning(self.h, arr, 64, ctypes.byref(n)))
        out = []
        for k in range(n.value):
            d = _struct_dict(arr[k])
            d["cls"] = f"({PAIR_CLASS[d['bra_class']]}|{PAIR_CLASS[d['ket_class']]})"
            out.append(d)
        return out

    def set_tuning(self, records):
        """Apply a list of tuning dicts (bra_class, ket_class, fp32, variant,
        waves_per_block[, ms])."""
        arr = (_Tuning * max(1, len(records)))()
        for k, r in enumerate(records):
            arr[k] = _Tuning(int(r["bra_class"]), int(r["ket_class"]), int(r["fp32"]),
                             int(r["variant"]), int(r["waves_per_block"]), 0, 0,
                             int(r.get("seg_tiles", 0)), float(r.get("ms", 0.0)))
        _check(lib().fsim_set_tuning(self.h, arr, len(records)))

    def set_all_variants(self, variant, waves_per_block=4):
        recs = [dict(bra_class=x, ket_class=y, fp32=f, variant=variant,
                     waves_per_block=waves_per_block)
                for x in range(6) for y in range(x + 1) for f in (0, 1)]
        self.set_tuning(recs)

    def autotune(self, D, precision="fp64"):
        _check(lib().fsim_autotune(self.h, _ptr(D), _PREC[precision], _stream()))
        return self.get_tuning()

    def eri_quartets(self, quartets, precision="fp64"):
        """Contracted Cartesian blocks (numpy) for an (n, 4) array of shell indices."""
        q = np.ascontiguousarray(quartets, dtype=np.int32).reshape(-1, 4)
        sizes = np.prod(np.array([[NCART[self.shell_l[s]] for s in row] for row in q]), axis=1) \
            if len(q) else np.zeros(0, dtype=np.int64)
        offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64) if len(q) else \
            np.zeros(0, dtype=np.int64)
        total = int(sizes.sum()) if len(q) else 0
        out = torch.full((max(total, 1),), float("nan"), dtype=torch.float64, device=self.device)
        _check(lib().fsim_eri_quartets(self.h, len(q), q.ctypes.data, offs.ctypes.data,
                                       _ptr(out), _PREC[precision], _stream()))
        torch.cuda.current_stream().synchronize()
        flat = out.cpu().numpy()
        blocks = []
        for k, row in enumerate(q):
            shp = tuple(NCART[self.shell_l[s]] for s in row)
            blocks.append(flat[offs[k]:offs[k] + sizes[k]].reshape(shp))
        return blocks

    def scf(self, precision="fp64", max_iter=100, D0=None, verbose=False, refine=True):
        """SCF driver: repeated fsim_scf_step until converged.  In mixed mode a
        final pure-FP64 Fock build at the converged density gives the
        reported energy (refinement)."""
        if self.screen_stats is None:
            self.schwarz_screen()
        self.scf_reset()
        D = self.core_guess() if D0 is None else D0.clone()
        hist = []
        info = None
        for _ in range(max_iter):
            Din = D.clone() if precision == "mixed" else None
            info = self.scf_step(D, precision)
            hist.append(info)
            if verbose:
                print(f"fsim scf {info['iter']:3d} E={info['E_total']:.12f} dE={info['dE']:.2e} "
                      f"rmsD={info['rms_dD']:.2e} diis={info['diis_used']}", flush=True)
            if info["converged"]:
                break
        res = {"E_total": info["E_total"], "iterations": info["iter"],
               "converged": bool(info["converged"]), "D": D, "history": hist}
        if precision == "mixed" and refine:
            # energy of the density the last step was given, from a pure FP64 build
            r = self.fock_build(Din, "fp64")
            res["E_total_mixed"] = info["E_total"]
            res["E_total"] = r["E_elec"] + self.enuc
        return res


class Batch(Context):
    """Many molecules in one context: every matrix is a packed 1-D tensor
    holding molecule m's N_m x N_m block at offsets[m]."""

    def __init__(self, bases, tau=0.0, tau_fp32=0.0, diis_m=8, conv_rms_dD=1e-8, conv_dE=1e-10,
                 max_iter=100, device="cuda"):
        L = lib()
        if not torch.cuda.is_available():
            raise FsimError("no GPU: libfsim runs on an MI355X only")
        self.device = torch.device(device)
        structs, keeps = [], []
        for b in bases:
            st, keep = basis_struct(b)
            structs.append(st)
            keeps.append(keep)
        arr = (_Basis * len(structs))(*structs)
        self.opt = _Options(float(tau), float(tau_fp32), int(diis_m), float(conv_rms_dD),
                            float(conv_dE), int(max_iter), 0)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(L.fsim_batch_create(arr, len(structs), ctypes.byref(self.opt), ctypes.byref(h)))
        self.h = h
        n, ns = ctypes.c_int32(), ctypes.c_int32()
        _check(L.fsim_nbf(self.h, ctypes.byref(n), ctypes.byref(ns)))
        self.nbf, self.nshell = n.value, ns.value
        self.nmol = len(bases)
        self.tau_prim = 0.0
        nm = ctypes.c_int32()
        self.nbf_mol = np.zeros(self.nmol, dtype=np.int32)
        self.offsets = np.zeros(self.nmol, dtype=np.int64)
        self.enuc_mol = np.zeros(self.nmol)
        packed = ctypes.c_int64()
        _check(L.fsim_batch_layout(self.h, ctypes.byref(nm), self.nbf_mol.ctypes.data,
                                   self.offsets.ctypes.data, self.enuc_mol.ctypes.data,
                                   ctypes.byref(packed)))
        self.packed = packed.value
        self.enuc = float(self.enuc_mol.sum())
        self.nelec = int(sum(int(b["nelec"]) for b in bases))
        self.tau, self.tau_fp32 = float(tau), float(tau_fp32)
        self.shell_l = np.concatenate([np.asarray(b["shell_l"], dtype=np.int32) for b in bases])
        self.screen_stats = None

    def _mat(self):
        return torch.empty(self.packed, dtype=torch.float64, device=self.device)

    def unpack(self, packed):
        return [packed[o:o + n * n].view(n, n) for o, n in zip(self.offsets, self.nbf_mol)]

    def pack(self, blocks):
        return torch.cat([b.reshape(-1) for b in blocks]).contiguous()

    def schwarz_screen(self, tau=None, tau_fp32=None, want_q=False):
        return super().schwarz_screen(tau, tau_fp32, want_q=False)

    def energies(self):
        E = np.zeros(self.nmol)
        _check(lib().fsim_batch_energies(self.h, E.ctypes.data))
        return E

    def scf_info(self):
        arr = (_ScfInfo * self.nmol)()
        _check(lib().fsim_batch_scf_info(self.h, arr))
        return [_struct_dict(arr[k]) for k in range(self.nmol)]


    def one_electron(self):
        S, H, X = self._mat(), self._mat(), self._mat()
        _check(lib().fsim_one_electron(self.h, _ptr(S), _ptr(H), _ptr(X), _stream()))
        return S, H, X

    def scf(self, precision="fp64", max_iter=100, D0=None, verbose=False, refine=True,
            stop_fraction=None):
        """All molecules at once; each molecule's energy and the iteration at
        which it first met the convergence test are returned.  stop_fraction:
        end as soon as that share of the molecules meets the test in the same
        step."""
        if self.screen_stats is None:
            self.schwarz_screen(want_q=False)
        self.scf_reset()
        D = self.core_guess() if D0 is None else D0.clone()
        first_conv = np.full(self.nmol, -1)
        info = None
        per = None
        Din = None
        for _ in range(max_iter):
            Din = D.clone() if precision == "mixed" else None
            info = self.scf_step(D, precision)
            per = self.scf_info()
            for m, r in enumerate(per):
                if r["converged"] and first_conv[m] < 0:
                    first_conv[m] = r["iter"]
            if verbose:
                print(f"fsim batch scf {info['iter']:3d} sumE={info['E_total']:.10f} "
                      f"max rmsD={info['rms_dD']:.2e} converged {int((first_conv >= 0).sum())}"
                      f"/{self.nmol}", flush=True)
            if info["converged"]:
                break
            if stop_fraction is not None and \
                    sum(1 for r in per if r["converged"]) >= stop_fraction * self.nmol:
                break
        E = np.array([r["E_total"] for r in per])
        res = {"E_total": E, "iterations": info["iter"], "converged": bool(info["converged"]),
               "first_converged": first_conv, "D": D, "per_molecule": per}
        if precision == "mixed" and refine:
            self.fock_build(Din, "fp64")
            res["E_total_mixed"] = E
            res["E_total"] = self.energies() + self.enuc_mol
        return res
