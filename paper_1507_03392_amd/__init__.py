"""Python binding of libecrpic (the MI355X ion PIC/MCC step behind include/ecrpic.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  PyTorch provides the device arena and the stream.
Importing this module does not need a GPU; creating a Run does, and raises
if the library is not built or no GPU is present.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libecrpic.so")

ABI_VERSION = 7
MAXS, MAXQ = 4, 32
MAXN = 4  # electrons one ionisation may remove
FPT_BINS = 32
BIRTH_NONE = 0xFFFFFFFF
FP64, FP32_MIXED = 0, 1
P_PUSH, P_IONIZE, P_CX, P_COULOMB, P_DEPOSIT, P_ALL, P_HEAT, P_ELASTIC = 1, 2, 4, 8, 16, 31, 32, 64
F_ION_N, F_ION_Q, F_ATOM_N, F_ION_P, N_FIELDS = 0, 1, 2, 3, 4
FLAG_EVENTS, FLAG_SPLIT, FLAG_SELF_NE, FLAG_HEAT_ISOTROPIC, FLAG_SELF_N0, FLAG_CX_PARTNER = 1, 2, 4, 8, 16, 32
K_SORT, K_COULOMB, K_PUSH, K_DEPOSIT, K_FUSED, K_COUL_PAIRS, K_PARTNER, K_STEP, N_KERNELS = 0, 1, 2, 3, 4, 5, 6, 7, 8
KERNEL_NAMES = ["sort", "coul_order", "push", "deposit", "push_deposit", "coul_pairs", "cx_partner", "step"]

STATUS = {0: "ECR_OK", -1: "ECR_EINVAL", -2: "ECR_ENOMEM", -3: "ECR_EDEVICE", -4: "ECR_ESTATE",
          -5: "ECR_ENUMERIC", -6: "ECR_EDT", -7: "ECR_EABI"}

EXPORTS = ["ecr_footprint", "ecr_create", "ecr_create_static", "ecr_init_ions", "ecr_step", "ecr_step_graph", "ecr_step_batch",
           "ecr_read_tallies", "ecr_read_density", "ecr_get_state", "ecr_set_state", "ecr_event_log", "ecr_weight", "ecr_profile", "ecr_profile_stride",
           "ecr_kernel_times", "ecr_last_error", "ecr_destroy", "ecr_selftest_philox", "ecr_selftest_divsqrt"]


class EcrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Species(C.Structure):
    _fields_ = [("mass_amu", C.c_double), ("z_max", C.c_int32), ("cx_forbidden_mask", C.c_uint32),
                ("fraction", C.c_double), ("k_ion_in_m3s", C.c_double * MAXQ),
                ("k_ion_out_m3s", C.c_double * MAXQ), ("sigma_cx1_m2", C.c_double), ("n0_m3", C.c_double),
                ("k_ion_multi_in_m3s", (C.c_double * MAXQ) * (MAXN - 1)),
                ("k_ion_multi_out_m3s", (C.c_double * MAXQ) * (MAXN - 1)), ("sigma_el1_m2", C.c_double)]


class Params(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("precision", C.c_int32), ("process_mask", C.c_uint32),
                ("deposit_mask", C.c_uint32), ("flags", C.c_uint32), ("sort_every", C.c_int32),
                ("seed", C.c_uint64), ("n_particles", C.c_int64), ("dt_s", C.c_double),
                ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("n_species", C.c_int32),
                ("R0_m", C.c_double), ("L_m", C.c_double), ("r_ap_m", C.c_double),
                ("inlet_x_m", C.c_double), ("inlet_y_m", C.c_double),
                ("B0_T", C.c_double), ("mirror_k", C.c_double), ("BH_T", C.c_double),
                ("zone_a_m", C.c_double), ("zone_c_m", C.c_double), ("ne_in_m3", C.c_double),
                ("ne_out_m3", C.c_double), ("Ti0_eV", C.c_double), ("T_wall_eV", C.c_double),
                ("T_n_eV", C.c_double), ("dE_cx_eV", C.c_double), ("lnL_ii", C.c_double),
                ("lnL_ei", C.c_double), ("Te_in_eV", C.c_double), ("Te_out_eV", C.c_double),
                ("weight", C.c_double), ("efield_nodes", C.POINTER(C.c_double)),
                ("bfield_nodes", C.POINTER(C.c_double)),
                ("species", Species * MAXS)]


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


class StateView(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("vx", C.c_void_p),
                ("vy", C.c_void_p), ("vz", C.c_void_p), ("q", C.c_void_p), ("species", C.c_void_p),
                ("cell", C.c_void_p), ("n", C.c_int64), ("step", C.c_int64), ("birth", C.c_void_p)]


_lib = None


def lib_available():
    return os.path.exists(LIB_PATH)


def lib():
    """Load libecrpic.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1507_03392_amd/build.py "
                               "(or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, u32, u64 = C.c_void_p, C.c_int64, C.c_int32, C.c_uint32, C.c_uint64
        sig = {
            "ecr_footprint": [C.POINTER(Params), C.POINTER(C.c_size_t)],
            "ecr_create": [C.POINTER(Params), vp, C.c_size_t, vp, C.POINTER(vp)],
            "ecr_create_static": [C.POINTER(Params), vp, C.POINTER(vp)],
            "ecr_init_ions": [vp], "ecr_step": [vp, i64], "ecr_step_graph": [vp, i64], "ecr_step_batch": [C.POINTER(vp), i32, i64, vp],
            "ecr_read_tallies": [vp, C.POINTER(Tallies)],
            "ecr_read_density": [vp, u32, vp, C.POINTER(i64)],
            "ecr_get_state": [vp, C.POINTER(StateView)], "ecr_set_state": [vp, C.POINTER(StateView)],
            "ecr_event_log": [vp, vp], "ecr_weight": [vp, C.POINTER(C.c_double)],
            "ecr_profile": [vp, i32], "ecr_profile_stride": [vp, i32], "ecr_kernel_times": [vp, vp, vp], "ecr_destroy": [vp],
            "ecr_selftest_philox": [u64, u32, u32, u32, u32, i64, vp, vp],
            "ecr_selftest_divsqrt": [vp, vp, i64, vp, vp, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.ecr_last_error.argtypes = [vp]
        L.ecr_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(st, handle=None):
    if st != 0:
        msg = lib().ecr_last_error(handle)
        raise EcrError(st, msg.decode() if msg else "")


def make_params(p, events=False, split=False):
    """Fill the library's ecr_params from a workload dict (SI units)."""
    P = Params()
    P.abi_version = ABI_VERSION
    P.precision = p.get("precision", FP64)
    P.process_mask = p["process_mask"]
    P.deposit_mask = p["deposit_mask"]
    P.flags = (FLAG_EVENTS if events else 0) | (FLAG_SPLIT if split else 0) | \
        (FLAG_SELF_NE if p.get("self_ne") else 0) | (FLAG_HEAT_ISOTROPIC if p.get("heat_isotropic") else 0) | \
        (FLAG_SELF_N0 if p.get("self_n0") else 0) | (FLAG_CX_PARTNER if p.get("cx_partner") else 0)
    P.sort_every = p["sort_every"]
    P.seed = p["seed"]
    P.n_particles = p["n"]
    P.dt_s = p["dt"]
    P.nx, P.ny, P.nz = p["nx"], p["ny"], p["nz"]
    P.n_species = len(p["species"])
    for dst, src in (("R0_m", "R0"), ("L_m", "L"), ("r_ap_m", "r_ap"), ("inlet_x_m", "inlet_x"),
                     ("inlet_y_m", "inlet_y"), ("B0_T", "B0"), ("mirror_k", "mirror_k"), ("BH_T", "BH"),
                     ("zone_a_m", "zone_a"), ("zone_c_m", "zone_c"), ("ne_in_m3", "ne_in"),
                     ("ne_out_m3", "ne_out"), ("Ti0_eV", "Ti0_eV"), ("T_wall_eV", "T_wall_eV"),
                     ("T_n_eV", "T_n_eV"), ("dE_cx_eV", "dE_cx_eV"), ("lnL_ii", "lnL"), ("weight", "weight")):
        setattr(P, dst, float(p[src]))
    P.lnL_ei = float(p.get("lnL_ei", 17.0))
    P.Te_in_eV = float(p.get("Te_in_eV", 0.0))
    P.Te_out_eV = float(p.get("Te_out_eV", 0.0))
    keep = None
    if p.get("efield") is not None or p.get("bfield") is not None:
        keep = []
    if p.get("efield") is not None:
        keep.append(np.ascontiguousarray(p["efield"], dtype=np.float64))
        P.efield_nodes = keep[-1].ctypes.data_as(C.POINTER(C.c_double))
    if p.get("bfield") is not None:
        keep.append(np.ascontiguousarray(p["bfield"], dtype=np.float64))
        P.bfield_nodes = keep[-1].ctypes.data_as(C.POINTER(C.c_double))
    for i, s in enumerate(p["species"]):
        S = P.species[i]
        S.mass_amu = s["mass_amu"]
        S.z_max = s["z_max"]
        S.cx_forbidden_mask = s["cx_forbidden_mask"]
        S.fraction = s["fraction"]
        for q in range(MAXQ):
            S.k_ion_in_m3s[q] = s["k_in"][q]
            S.k_ion_out_m3s[q] = s["k_out"][q]
        S.sigma_cx1_m2 = s["sigma_cx1"]
        S.n0_m3 = s["n0"]
        for key, dst in (("k_multi_in", S.k_ion_multi_in_m3s), ("k_multi_out", S.k_ion_multi_out_m3s)):
            tab = s.get(key)
            if tab is not None:
                for j in range(MAXN - 1):
                    for q in range(MAXQ):
                        dst[j][q] = tab[j][q]
        S.sigma_el1_m2 = s.get("sigma_el1", 0.0)
    return P, keep


def footprint(params, events=False):
    P, _keep = make_params(params, events)
    n = C.c_size_t()
    _check(lib().ecr_footprint(C.byref(P), C.byref(n)))
    return n.value


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def tallies_to_dict(t):
    g = lambda a: np.array([a[s][:] for s in range(MAXS)], dtype=np.uint64)
    d = lambda a: np.array([a[s][:] for s in range(MAXS)], dtype=np.float64)
    return dict(extracted=g(t.extracted), wall=g(t.wall), ionized=g(t.ionized), cx=g(t.cx),
                cx_products=np.array(t.cx_products[:], dtype=np.uint64), recycled=int(t.recycled),
                anomalies=int(t.anomalies), steps=int(t.steps), coul_dp=np.array(t.coul_dp[:]),
                coul_de=float(t.coul_de), coul_e=float(t.coul_e), fpt_n=g(t.fpt_n), fpt_sum=g(t.fpt_sum),
                fpt_hist=g(t.fpt_hist), extracted_r=d(t.extracted_r), lost_ke=np.array(t.lost_ke[:]),
                ionized_n=g(t.ionized_n), elastic=g(t.elastic),
                cx_unmatched=np.array(t.cx_unmatched[:], dtype=np.uint64))


class Run:
    """One simulation run on the GPU: arena and stream from torch, all compute in libecrpic."""

    def __init__(self, params, events=False, split=False, device=None, stream=None, arena=None, static=False):
        """static=True: the run lives in the library's static device
        workspace (ecr_create_static, no device allocation); else in an arena
        from torch (or the given one)."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the ion step runs only in the HIP library")
        self.params = params
        self.n = params["n"]
        self.nnode = (params["nx"] + 1) * (params["ny"] + 1) * (params["nz"] + 1)
        self.events_enabled = events
        P, keep = make_params(params, events, split)
        nbytes = C.c_size_t()
        _check(lib().ecr_footprint(C.byref(P), C.byref(nbytes)))
        self.nbytes = nbytes.value
        dev = torch.device(device or "cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = C.c_void_p()
        if static:
            self.arena = None
            with torch.cuda.device(dev):
                _check(lib().ecr_create_static(C.byref(P), C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        else:
            self.arena = arena if arena is not None else torch.empty(self.nbytes, dtype=torch.uint8, device=dev)
            _check(lib().ecr_create(C.byref(P), C.c_void_p(self.arena.data_ptr()), self.nbytes,
                                    C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        del keep
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().ecr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_ions(self):
        _check(lib().ecr_init_ions(self.h), self.h)

    def step(self, n=1):
        _check(lib().ecr_step(self.h, int(n)), self.h)

    def step_graph(self, n):
        """n steps; whole sort periods replay a captured HIP graph."""
        _check(lib().ecr_step_graph(self.h, int(n)), self.h)

    def tallies(self, allow_anomalies=True):
        t = Tallies()
        st = lib().ecr_read_tallies(self.h, C.byref(t))
        if st != 0 and not (allow_anomalies and st == -5):
            _check(st, self.h)
        return tallies_to_dict(t)

    def density(self, field):
        out = np.empty(self.nnode, dtype=np.float64)
        steps = C.c_int64()
        _check(lib().ecr_read_density(self.h, field, _ptr(out), C.byref(steps)), self.h)
        return out, steps.value

    def get_state(self):
        n = self.n
        out = {k: np.empty(n, dtype=np.float64) for k in ("x", "y", "z", "vx", "vy", "vz")}
        out["q"] = np.empty(n, dtype=np.uint8)
        out["species"] = np.empty(n, dtype=np.uint8)
        out["cell"] = np.empty(n, dtype=np.uint32)
        out["birth"] = np.empty(n, dtype=np.uint32)
        v = StateView(*(_ptr(out[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "q", "species", "cell")), n, 0,
                      _ptr(out["birth"]))
        _check(lib().ecr_get_state(self.h, C.byref(v)), self.h)
        out["step"] = v.step
        return out

    def set_state(self, st, step=0, cell=None):
        a = {k: np.ascontiguousarray(st[k], dtype=np.float64) for k in ("x", "y", "z", "vx", "vy", "vz")}
        q = np.ascontiguousarray(st["q"], dtype=np.uint8)
        c = None if cell is None else np.ascontiguousarray(cell, dtype=np.uint32)
        b = np.ascontiguousarray(st["birth"], dtype=np.uint32) if st.get("birth") is not None else None
        v = StateView(*(_ptr(a[k]) for k in ("x", "y", "z", "vx", "vy", "vz")), _ptr(q), None, _ptr(c),
                      self.n, int(step), _ptr(b))
        _check(lib().ecr_set_state(self.h, C.byref(v)), self.h)

    def events(self):
        out = np.empty(self.n, dtype=np.uint8)
        _check(lib().ecr_event_log(self.h, _ptr(out)), self.h)
        return out

    @property
    def weight(self):
        w = C.c_double()
        _check(lib().ecr_weight(self.h, C.byref(w)), self.h)
        return w.value

    def profile(self, enable=True, kinds=None, stride=1):
        """Time launches with HIP events: every kernel kind, or only `kinds`
        (names from KERNEL_NAMES), one launch in `stride` of each; enable=False
        turns timing off."""
        mask = 0
        if enable:
            mask = -1 if kinds is None else sum(1 << KERNEL_NAMES.index(k) for k in kinds)
        _check(lib().ecr_profile_stride(self.h, stride), self.h)
        _check(lib().ecr_profile(self.h, mask), self.h)

    def kernel_times(self):
        ms = np.zeros(N_KERNELS)
        cnt = np.zeros(N_KERNELS, dtype=np.int64)
        _check(lib().ecr_kernel_times(self.h, _ptr(ms), _ptr(cnt)), self.h)
        return {KERNEL_NAMES[k]: (float(ms[k]), int(cnt[k])) for k in range(N_KERNELS)}


def step_batch(runs, n_steps, stream):
    arr = (C.c_void_p * len(runs))(*[r.h for r in runs])
    _check(lib().ecr_step_batch(arr, len(runs), int(n_steps), C.c_void_p(stream.cuda_stream)))


def selftest_philox(seed, ctr0, c1, c2, c3, n):
    import torch
    out = torch.empty(4 * n, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream()
    _check(lib().ecr_selftest_philox(seed, ctr0, c1, c2, c3, n, C.c_void_p(out.data_ptr()),
                                     C.c_void_p(s.cuda_stream)))
    s.synchronize()
    return out.cpu().numpy().view(np.uint32).reshape(n, 4)


def selftest_divsqrt(a, b):
    import torch
    ta = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    tb = torch.from_numpy(np.ascontiguousarray(b, dtype=np.float64)).cuda()
    q = torch.empty_like(ta)
    r = torch.empty_like(ta)
    s = torch.cuda.current_stream()
    _check(lib().ecr_selftest_divsqrt(C.c_void_p(ta.data_ptr()), C.c_void_p(tb.data_ptr()), ta.numel(),
                                      C.c_void_p(q.data_ptr()), C.c_void_p(r.data_ptr()), C.c_void_p(s.cuda_stream)))
    s.synchronize()
    return q.cpu().numpy(), r.cpu().numpy()
