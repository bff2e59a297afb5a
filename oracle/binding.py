"""ctypes binding of the CPU oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libecr_oracle.so")

MAXS, MAXQ = 4, 32
MAXN = 4
FPT_BINS = 32
BIRTH_NONE = 0xFFFFFFFF


class Species(C.Structure):
    _fields_ = [("mass_amu", C.c_double), ("z_max", C.c_int32), ("cx_forbidden_mask", C.c_uint32),
                ("fraction", C.c_double), ("k_in", C.c_double * MAXQ), ("k_out", C.c_double * MAXQ),
                ("sigma_cx1", C.c_double), ("n0", C.c_double),
                ("k_multi_in", (C.c_double * MAXQ) * (MAXN - 1)), ("k_multi_out", (C.c_double * MAXQ) * (MAXN - 1)),
                ("sigma_el1", C.c_double)]


class Params(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("n", C.c_int64), ("dt", C.c_double), ("sort_every", C.c_int32),
                ("process_mask", C.c_uint32), ("deposit_mask", C.c_uint32),
                ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("R0", C.c_double), ("L", C.c_double), ("r_ap", C.c_double),
                ("inlet_x", C.c_double), ("inlet_y", C.c_double),
                ("B0", C.c_double), ("mirror_k", C.c_double), ("BH", C.c_double),
                ("zone_a", C.c_double), ("zone_c", C.c_double), ("ne_in", C.c_double), ("ne_out", C.c_double),
                ("Ti0_eV", C.c_double), ("T_wall_eV", C.c_double), ("T_n_eV", C.c_double),
                ("dE_cx_eV", C.c_double), ("lnL", C.c_double), ("weight", C.c_double),
                ("efield", C.POINTER(C.c_double)), ("n_species", C.c_int32),
                ("sp", Species * MAXS), ("self_ne", C.c_int32),
                ("lnL_ei", C.c_double), ("Te_in_eV", C.c_double), ("Te_out_eV", C.c_double),
                ("bfield", C.POINTER(C.c_double)), ("heat_isotropic", C.c_int32),
                ("self_n0", C.c_int32), ("cx_partner", C.c_int32)]


class Tallies(C.Structure):
    _fields_ = [("extracted", (C.c_uint64 * MAXQ) * MAXS), ("wall", (C.c_uint64 * MAXQ) * MAXS),
                ("ionized", (C.c_uint64 * MAXQ) * MAXS), ("cx", (C.c_uint64 * MAXQ) * MAXS),
                ("cx_products", C.c_uint64 * MAXS), ("recycled", C.c_uint64), ("anomalies", C.c_uint64),
                ("steps", C.c_int64), ("coul_dp", C.c_double * 3), ("coul_de", C.c_double),
                ("coul_e", C.c_double), ("fpt_n", (C.c_uint64 * MAXQ) * MAXS),
                ("fpt_sum", (C.c_uint64 * MAXQ) * MAXS), ("fpt_hist", (C.c_uint64 * FPT_BINS) * MAXS),
                ("extracted_r", (C.c_double * MAXQ) * MAXS), ("lost_ke", C.c_double * MAXS),
                ("ionized_n", (C.c_uint64 * MAXN) * MAXS), ("elastic", (C.c_uint64 * MAXQ) * MAXS),
                ("cx_unmatched", C.c_uint64 * MAXS)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.orc_create.argtypes = [C.POINTER(Params), C.POINTER(C.c_void_p)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_init_ions.argtypes = [C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_set_state.argtypes = [C.c_void_p, C.c_int64] + [C.c_void_p] * 9
        L.orc_get_state.argtypes = [C.c_void_p, C.POINTER(C.c_int64)] + [C.c_void_p] * 10
        L.orc_get_tallies.argtypes = [C.c_void_p, C.POINTER(Tallies)]
        L.orc_get_density.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.POINTER(C.c_int64)]
        L.orc_get_events.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_weight.argtypes = [C.c_void_p]
        L.orc_weight.restype = C.c_double
        L.orc_philox4x32_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_philox4x64_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_u53.argtypes = [C.c_uint32, C.c_uint32]
        L.orc_u53.restype = C.c_double
        L.orc_field.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, dp]
        L.orc_boris.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, dp, dp]
        L.orc_nanbu_A.argtypes = [C.c_void_p, C.c_double]
        L.orc_nanbu_A.restype = C.c_double
        L.orc_nanbu_A_root.argtypes = [C.c_double]
        L.orc_nanbu_A_root.restype = C.c_double
        L.orc_nanbu_omc.argtypes = [C.c_void_p, C.c_double, C.c_double]
        L.orc_nanbu_omc.restype = C.c_double
        L.orc_segment_exit.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_segment_exit.restype = C.c_int
        L.orc_cell_of.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double]
        L.orc_cell_of.restype = C.c_uint32
        L.orc_set_ids.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_philox_fill.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int64,
                                      C.c_void_p]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def make_params(p):
    """Fill the oracle's own parameter struct from a workload dict."""
    P = Params()
    P.seed = p["seed"]
    P.n = p["n"]
    P.dt = p["dt"]
    P.sort_every = p["sort_every"]
    P.process_mask = p["process_mask"]
    P.deposit_mask = p["deposit_mask"]
    P.nx, P.ny, P.nz = p["nx"], p["ny"], p["nz"]
    for k in ("R0", "L", "r_ap", "inlet_x", "inlet_y", "B0", "mirror_k", "BH", "zone_a", "zone_c",
              "ne_in", "ne_out", "Ti0_eV", "T_wall_eV", "T_n_eV", "dE_cx_eV", "lnL", "weight"):
        setattr(P, k, float(p[k]))
    keep = []
    if p.get("efield") is not None:
        keep.append(np.ascontiguousarray(p["efield"], dtype=np.float64))
        P.efield = keep[-1].ctypes.data_as(C.POINTER(C.c_double))
    if p.get("bfield") is not None:
        keep.append(np.ascontiguousarray(p["bfield"], dtype=np.float64))
        P.bfield = keep[-1].ctypes.data_as(C.POINTER(C.c_double))
    P.n_species = len(p["species"])
    for i, s in enumerate(p["species"]):
        S = P.sp[i]
        S.mass_amu = s["mass_amu"]
        S.z_max = s["z_max"]
        S.cx_forbidden_mask = s["cx_forbidden_mask"]
        S.fraction = s["fraction"]
        for q in range(MAXQ):
            S.k_in[q] = s["k_in"][q]
            S.k_out[q] = s["k_out"][q]
        S.sigma_cx1 = s["sigma_cx1"]
        S.n0 = s["n0"]
        for k in ("k_multi_in", "k_multi_out"):
            tab = s.get(k)
            if tab is not None:
                for j in range(MAXN - 1):
                    for q in range(MAXQ):
                        getattr(S, k)[j][q] = tab[j][q]
        S.sigma_el1 = s.get("sigma_el1", 0.0)
    P.self_ne = 1 if p.get("self_ne") else 0
    P.lnL_ei = float(p.get("lnL_ei", 17.0))
    P.heat_isotropic = 1 if p.get("heat_isotropic") else 0
    P.self_n0 = 1 if p.get("self_n0") else 0
    P.cx_partner = 1 if p.get("cx_partner") else 0
    P.Te_in_eV = float(p.get("Te_in_eV", 0.0))
    P.Te_out_eV = float(p.get("Te_out_eV", 0.0))
    return P, keep


class OracleSim:
    """One oracle run: create, init or set state, step, read back."""

    def __init__(self, params):
        self.params = params
        self._P, self._keep = make_params(params)
        h = C.c_void_p()
        rc = lib().orc_create(C.byref(self._P), C.byref(h))
        if rc != 0:
            raise ValueError(f"orc_create failed ({rc})")
        self.h = h
        self.n = params["n"]
        nx, ny, nz = params["nx"], params["ny"], params["nz"]
        self.nnode = (nx + 1) * (ny + 1) * (nz + 1)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    def init_ions(self):
        lib().orc_init_ions(self.h)

    def set_ids(self, ids, species):
        a = np.ascontiguousarray(ids, dtype=np.uint32)
        b = np.ascontiguousarray(species, dtype=np.uint8)
        if lib().orc_set_ids(self.h, _ptr(a), _ptr(b)) != 0:
            raise ValueError("bad species")

    def step(self, n=1):
        lib().orc_step(self.h, n)

    def set_state(self, st, step=0, cell=None):
        a = {k: np.ascontiguousarray(st[k], dtype=np.float64) for k in ("x", "y", "z", "vx", "vy", "vz")}
        q = np.ascontiguousarray(st["q"], dtype=np.uint8)
        c = None if cell is None else np.ascontiguousarray(cell, dtype=np.uint32)
        b = np.ascontiguousarray(st["birth"], dtype=np.uint32) if st.get("birth") is not None else None
        rc = lib().orc_set_state(self.h, step, _ptr(a["x"]), _ptr(a["y"]), _ptr(a["z"]), _ptr(a["vx"]),
                                 _ptr(a["vy"]), _ptr(a["vz"]), _ptr(q), _ptr(c), _ptr(b))
        if rc != 0:
            raise ValueError(f"orc_set_state failed ({rc})")

    def get_state(self):
        n = self.n
        out = {k: np.empty(n, dtype=np.float64) for k in ("x", "y", "z", "vx", "vy", "vz")}
        out["q"] = np.empty(n, dtype=np.uint8)
        out["species"] = np.empty(n, dtype=np.uint8)
        out["cell"] = np.empty(n, dtype=np.uint32)
        step = C.c_int64()
        out["birth"] = np.empty(n, dtype=np.uint32)
        lib().orc_get_state(self.h, C.byref(step), _ptr(out["x"]), _ptr(out["y"]), _ptr(out["z"]),
                            _ptr(out["vx"]), _ptr(out["vy"]), _ptr(out["vz"]), _ptr(out["q"]),
                            _ptr(out["species"]), _ptr(out["cell"]), _ptr(out["birth"]))
        out["step"] = step.value
        return out

    def tallies(self):
        t = Tallies()
        lib().orc_get_tallies(self.h, C.byref(t))
        return tallies_to_dict(t)

    def density(self, field):
        out = np.empty(self.nnode, dtype=np.float64)
        steps = C.c_int64()
        if lib().orc_get_density(self.h, field, _ptr(out), C.byref(steps)) != 0:
            raise ValueError("bad field")
        return out, steps.value

    def events(self):
        out = np.empty(self.n, dtype=np.uint8)
        lib().orc_get_events(self.h, _ptr(out))
        return out

    @property
    def weight(self):
        return lib().orc_weight(self.h)

    # unit entry points
    def field(self, x, y, z):
        B = (C.c_double * 3)()
        lib().orc_field(self.h, x, y, z, B)
        return np.array(B[:])

    def boris(self, species, q, x, v, E=None):
        xa = (C.c_double * 3)(*x)
        va = (C.c_double * 3)(*v)
        Ea = None if E is None else C.cast((C.c_double * 3)(*E), C.c_void_p)
        lib().orc_boris(self.h, species, q, Ea, xa, va)
        return np.array(xa[:]), np.array(va[:])

    def nanbu_A(self, s):
        return lib().orc_nanbu_A(self.h, s)

    def nanbu_omc(self, s, u):
        return lib().orc_nanbu_omc(self.h, s, u)

    def segment_exit(self, x0, x1):
        a = (C.c_double * 3)(*x0)
        b = (C.c_double * 3)(*x1)
        f = C.c_double()
        k = lib().orc_segment_exit(self.h, a, b, C.byref(f))
        return k, f.value

    def cell_of(self, x, y, z):
        return lib().orc_cell_of(self.h, x, y, z)


def nanbu_A_root(s):
    return lib().orc_nanbu_A_root(s)


def philox4x32(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return list(o)


def philox4x64(ctr, key):
    c = (C.c_uint64 * 4)(*ctr)
    k = (C.c_uint64 * 2)(*key)
    o = (C.c_uint64 * 4)()
    lib().orc_philox4x64_10(c, k, o)
    return list(o)


def u53(a, b):
    return lib().orc_u53(a, b)


def philox_fill(seed, ctr0, c1, c2, c3, n):
    out = np.empty(4 * n, dtype=np.uint32)
    lib().orc_philox_fill(seed, ctr0, c1, c2, c3, n, _ptr(out))
    return out.reshape(n, 4)


def tallies_to_dict(t):
    return dict(
        extracted=np.array([[t.extracted[s][q] for q in range(MAXQ)] for s in range(MAXS)], dtype=np.uint64),
        wall=np.array([[t.wall[s][q] for q in range(MAXQ)] for s in range(MAXS)], dtype=np.uint64),
        ionized=np.array([[t.ionized[s][q] for q in range(MAXQ)] for s in range(MAXS)], dtype=np.uint64),
        cx=np.array([[t.cx[s][q] for q in range(MAXQ)] for s in range(MAXS)], dtype=np.uint64),
        cx_products=np.array(t.cx_products[:], dtype=np.uint64),
        recycled=int(t.recycled), anomalies=int(t.anomalies), steps=int(t.steps),
        coul_dp=np.array(t.coul_dp[:]), coul_de=float(t.coul_de), coul_e=float(t.coul_e),
        fpt_n=np.array([t.fpt_n[s][:] for s in range(MAXS)], dtype=np.uint64),
        fpt_sum=np.array([t.fpt_sum[s][:] for s in range(MAXS)], dtype=np.uint64),
        fpt_hist=np.array([t.fpt_hist[s][:] for s in range(MAXS)], dtype=np.uint64),
        extracted_r=np.array([t.extracted_r[s][:] for s in range(MAXS)], dtype=np.float64),
        lost_ke=np.array(t.lost_ke[:], dtype=np.float64),
        ionized_n=np.array([t.ionized_n[s][:] for s in range(MAXS)], dtype=np.uint64),
        elastic=np.array([t.elastic[s][:] for s in range(MAXS)], dtype=np.uint64),
        cx_unmatched=np.array(t.cx_unmatched[:], dtype=np.uint64))
