"""FP64 CPU oracle for linked-cell LJ + ATM forces.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.  It shares no
code with the GPU path.  The compiled part is ``atm3_oracle.c`` (plain C, FP64,
OpenMP), built into ``liboracle.so`` next to this file; ``surrogate.py`` is the FP64
numpy reference of the learned pair model.

Citations refer to "Linked Cell Traversal Algorithms for Three-Body
Interactions in Molecular Dynamics": Sec. 2 (truncation rules, eqs. forcepairs,
atm, ATMGradient), Sec. 3 (eqs. celltriplet, twoonetriplets, carttriplets,
totalInteractions), Sec. 4 (traversals 3c01/3c18/3c08), Sec. 5 (LJ in reduced
units, eq. P_3).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "atm3_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

TRUNCATIONS = {"pair": 0, "product": 1}
VARIANTS = {"3c08": 0, "3c18": 1, "3c01": 2}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
            "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("sigma", ctypes.c_double),
                ("nu", ctypes.c_double), ("rc", ctypes.c_double),
                ("truncation", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("terms", ctypes.c_int32), ("pad", ctypes.c_int32)]


class _Result(ctypes.Structure):
    _fields_ = [("e_lj", ctypes.c_double), ("e_atm", ctypes.c_double),
                ("w_lj", ctypes.c_double), ("w_atm", ctypes.c_double),
                ("n_pairs", ctypes.c_int64), ("n_triplets", ctypes.c_int64),
                ("n_candidates", ctypes.c_int64), ("n_distinct", ctypes.c_int64)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        lib.orc_grid.argtypes = [P(ctypes.c_double), ctypes.c_double, P(ctypes.c_int32)]
        lib.orc_grid.restype = ctypes.c_int
        lib.orc_bin.argtypes = [P(ctypes.c_double), ctypes.c_int64, P(ctypes.c_double),
                                P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_int32)]
        lib.orc_bin.restype = None
        lib.orc_atm_energy.argtypes = [ctypes.c_double] * 4
        lib.orc_atm_energy.restype = ctypes.c_double
        lib.orc_atm_dudr.argtypes = [ctypes.c_double] * 4
        lib.orc_atm_dudr.restype = ctypes.c_double
        lib.orc_brute.argtypes = [P(ctypes.c_double), ctypes.c_int64, P(ctypes.c_double),
                                  P(_Params), P(ctypes.c_double), P(_Result)]
        lib.orc_brute.restype = ctypes.c_int
        lib.orc_brute_tensor.argtypes = lib.orc_brute.argtypes + [P(ctypes.c_double)]
        lib.orc_brute_tensor.restype = ctypes.c_int
        lib.orc_molecules.argtypes = [P(ctypes.c_double), ctypes.c_int64, P(ctypes.c_double),
                                      P(_Params), P(ctypes.c_int64), ctypes.c_int64,
                                      P(ctypes.c_double), P(_Result)]
        lib.orc_molecules.restype = ctypes.c_int
        lib.orc_triplet.argtypes = [P(ctypes.c_double)] * 3 + [ctypes.c_double] + \
            [P(ctypes.c_double)] * 3 + [P(ctypes.c_double)] * 2
        lib.orc_triplet.restype = None
        lib.orc_visited.argtypes = [P(ctypes.c_int32)] * 4 + [ctypes.c_int]
        lib.orc_visited.restype = ctypes.c_int
        lib.orc_cells.argtypes = [P(ctypes.c_double), ctypes.c_int64, P(ctypes.c_double), P(_Params),
                                  ctypes.c_int64, ctypes.c_int64, P(ctypes.c_double), P(_Result)]
        lib.orc_cells.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_set_threads.restype = None
        lib.orc_threads.argtypes = []
        lib.orc_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


@dataclass
class Result:
    """Outputs of one oracle evaluation (energies in eps, virial W = sum r.F)."""
    forces: np.ndarray
    e_lj: float
    e_atm: float
    w_lj: float
    w_atm: float
    n_pairs: int
    n_triplets: int
    n_candidates: int
    n_distinct: int = -1  # included triplets counted once (brute force only)


def _params(rc, nu, eps, sigma, truncation, variant, terms):
    return _Params(float(eps), float(sigma), float(nu), float(rc),
                   TRUNCATIONS[truncation], VARIANTS[variant], int(terms), 0)


def grid(box, rc):
    """Cells per dimension, floor(L_d / rc) (Sec. 4: cell side >= rc)."""
    lib = _load()
    b = np.ascontiguousarray(box, dtype=np.float64)
    n = np.zeros(3, dtype=np.int32)
    if lib.orc_grid(_dp(b), float(rc), _ip(n)) != 0:
        raise ValueError("invalid box / rc")
    return n


def bin_cells(pos, box, rc):
    """Per-molecule cell coordinates (N,3) and lexicographic linear index (N,)."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    b = np.ascontiguousarray(box, dtype=np.float64)
    n = grid(b, rc)
    cxyz = np.zeros((len(pos), 3), dtype=np.int32)
    clin = np.zeros(len(pos), dtype=np.int32)
    lib.orc_bin(_dp(pos), len(pos), _dp(b), _ip(n), _ip(cxyz), _ip(clin))
    return cxyz, clin, n


def brute(pos, box, rc=2.5, nu=0.073, eps=1.0, sigma=1.0, truncation="pair",
          variant="3c08", terms=3) -> Result:
    """O(N^3) evaluation of every pair and triplet under the inclusion rule."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    b = np.ascontiguousarray(box, dtype=np.float64)
    f = np.zeros_like(pos)
    r = _Result()
    p = _params(rc, nu, eps, sigma, truncation, variant, terms)
    if lib.orc_brute(_dp(pos), len(pos), _dp(b), ctypes.byref(p), _dp(f), ctypes.byref(r)) != 0:
        raise ValueError("oracle: invalid arguments")
    return Result(f, r.e_lj, r.e_atm, r.w_lj, r.w_atm, r.n_pairs, r.n_triplets, r.n_candidates, r.n_distinct)


def virial_diag(pos, box, rc=2.5, nu=0.073, eps=1.0, sigma=1.0, truncation="pair",
                variant="3c08", terms=3):
    """Diagonal of the virial tensor, W_aa = sum over force pairs of r_a F_a,
    for LJ and for ATM (the three force pairs of eq. (forcepairs) of every
    included triplet), by the O(N^3) evaluation; returns (w_lj[3], w_atm[3],
    Result)."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    b = np.ascontiguousarray(box, dtype=np.float64)
    f = np.zeros_like(pos)
    r = _Result()
    w = np.zeros(6)
    p = _params(rc, nu, eps, sigma, truncation, variant, terms)
    if lib.orc_brute_tensor(_dp(pos), len(pos), _dp(b), ctypes.byref(p), _dp(f), ctypes.byref(r), _dp(w)) != 0:
        raise ValueError("oracle: invalid arguments")
    res = Result(f, r.e_lj, r.e_atm, r.w_lj, r.w_atm, r.n_pairs, r.n_triplets, r.n_candidates, r.n_distinct)
    return w[:3].copy(), w[3:].copy(), res


def molecules(pos, box, rc=2.5, nu=0.073, eps=1.0, sigma=1.0, truncation="pair",
              variant="3c08", terms=3, sample=None) -> Result:
    """Per-molecule evaluation: forces of the sampled molecules (all if None);
    totals are whole-system values only when ``sample`` is None."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    b = np.ascontiguousarray(box, dtype=np.float64)
    p = _params(rc, nu, eps, sigma, truncation, variant, terms)
    r = _Result()
    if sample is None:
        f = np.zeros_like(pos)
        rc_ = lib.orc_molecules(_dp(pos), len(pos), _dp(b), ctypes.byref(p), None, 0,
                                _dp(f), ctypes.byref(r))
    else:
        s = np.ascontiguousarray(sample, dtype=np.int64)
        f = np.zeros((len(s), 3), dtype=np.float64)
        rc_ = lib.orc_molecules(_dp(pos), len(pos), _dp(b), ctypes.byref(p),
                                s.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(s),
                                _dp(f), ctypes.byref(r))
    if rc_ != 0:
        raise ValueError("oracle: invalid arguments")
    return Result(f, r.e_lj, r.e_atm, r.w_lj, r.w_atm, r.n_pairs, r.n_triplets, r.n_candidates, r.n_distinct)


def cells(pos, box, rc=2.5, nu=0.073, eps=1.0, sigma=1.0, terms=3, base_cells=None) -> Result:
    """Linked-cell evaluation with Newton 3 over the 3c08 cell sets, pairwise
    cutoff (the CPU counterpart of the method's structure, for timing).
    ``base_cells=(b0, b1)`` restricts it to that range of base cells."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    b = np.ascontiguousarray(box, dtype=np.float64)
    f = np.zeros_like(pos)
    r = _Result()
    p = _params(rc, nu, eps, sigma, "pair", "3c08", terms)
    b0, b1 = base_cells if base_cells is not None else (0, 0)
    if lib.orc_cells(_dp(pos), len(pos), _dp(b), ctypes.byref(p), int(b0), int(b1), _dp(f), ctypes.byref(r)) != 0:
        raise ValueError("oracle: invalid arguments (pairwise cutoff, >= 3 cells per dimension)")
    return Result(f, r.e_lj, r.e_atm, r.w_lj, r.w_atm, r.n_pairs, r.n_triplets, r.n_candidates, r.n_distinct)


def set_threads(k: int) -> None:
    """Number of OpenMP threads for the oracle's parallel loops."""
    _load().orc_set_threads(int(k))


def threads() -> int:
    """OpenMP threads the oracle uses."""
    return int(_load().orc_threads())


def atm_energy(rij, rik, rjk, nu):
    """eq. (atm) for side lengths."""
    return _load().orc_atm_energy(float(rij), float(rik), float(rjk), float(nu))


def atm_dudr(a, b, c, nu):
    """eq. (ATMGradient): du/d(side a) with b, c the other two sides."""
    return _load().orc_atm_dudr(float(a), float(b), float(c), float(nu))


def triplet(rij, rik, rjk, nu):
    """Forces on i, j, k (eq. forcepairs), energy and virial of one triplet."""
    lib = _load()
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (rij, rik, rjk)]
    fi, fj, fk = (np.zeros(3) for _ in range(3))
    u = ctypes.c_double()
    w = ctypes.c_double()
    lib.orc_triplet(_dp(a[0]), _dp(a[1]), _dp(a[2]), float(nu), _dp(fi), _dp(fj), _dp(fk),
                    ctypes.byref(u), ctypes.byref(w))
    return fi, fj, fk, u.value, w.value


def visited(ci, cj, ck, ncell, variant):
    """Visited-set predicate for three cells (3c01: mask of receiving molecules)."""
    a = [np.ascontiguousarray(v, dtype=np.int32) for v in (ci, cj, ck, ncell)]
    return _load().orc_visited(_ip(a[0]), _ip(a[1]), _ip(a[2]), _ip(a[3]), VARIANTS[variant])
