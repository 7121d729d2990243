"""ctypes wrapper of the C oracle (pd_oracle.c) -- TEST INFRASTRUCTURE.

Argument marshalling only; every computation is in pd_oracle.c.  Only the
tests, the smoke check and the CPU-baseline leg of the benchmark use it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pd_oracle.c")


def oracle_library_path(openmp: bool = True) -> str:
    return os.path.join(_HERE, "libpd_oracle_omp.so" if openmp else "libpd_oracle.so")


def build_oracle(force: bool = True) -> list:
    """Compile the oracle with gcc (FP64, no contraction, no fast-math)."""
    outs = []
    for omp in (False, True):
        out = oracle_library_path(omp)
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
            cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-shared",
                   "-fPIC", "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", out + ".tmp", "-lm"]
            if omp:
                cmd.insert(1, "-fopenmp")
            subprocess.run(cmd, check=True)
            os.replace(out + ".tmp", out)
        outs.append(out)
    return outs


class _Material(C.Structure):
    _fields_ = [("rho", C.c_double), ("bulk_k", C.c_double), ("young_E", C.c_double),
                ("Gc", C.c_double), ("horizon", C.c_double), ("micro", C.c_int32)]


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class _Problem(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_particles", C.c_int32), ("n_aggregates", C.c_int32),
                ("n_materials", C.c_int32),
                ("x", _dp), ("y", _dp), ("vol", _dp),
                ("particle_offset", _ip), ("particle_material", _ip), ("particle_aggregate", _ip),
                ("materials", C.POINTER(_Material)),
                ("loop_offset", _ip), ("loop_vertex_offset", _ip), ("loop_xy", _dp),
                ("u0x", _dp), ("u0y", _dp), ("v0x", _dp), ("v0y", _dp),
                ("contact_radius", C.c_double), ("friction_mu", C.c_double),
                ("damping_ratio", C.c_double), ("kn_mode", C.c_int32),
                ("box", _dp), ("top_wall_speed", _dp),
                ("gravity_x", C.c_double), ("gravity_y", C.c_double), ("dt", C.c_double),
                ("contact_mode", C.c_int32), ("n_threads", C.c_int32)]


_LIBS: dict = {}


def _lib(openmp: bool):
    key = bool(openmp)
    if key not in _LIBS:
        path = oracle_library_path(openmp)
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build_oracle(force=False)
        L = C.CDLL(path)
        vp = C.c_void_p
        L.or_create.argtypes = [C.POINTER(_Problem), C.POINTER(vp)]
        L.or_destroy.argtypes = [vp]
        L.or_error.argtypes = [vp]
        L.or_error.restype = C.c_char_p
        L.or_constants.argtypes = [vp, _dp]
        L.or_n_bonds.argtypes = [vp]
        L.or_n_bonds.restype = C.c_int64
        L.or_bonds.argtypes = [vp, _ip, _ip]
        L.or_step.argtypes = [vp, C.c_int64]
        L.or_forces.argtypes = [vp, C.c_uint32, _dp, _dp]
        L.or_damage.argtypes = [vp, _dp, C.POINTER(C.c_int64)]
        L.or_contacts.argtypes = [vp, _ip, _ip, C.c_int64]
        L.or_contacts.restype = C.c_int64
        L.or_get_state.argtypes = [vp, _dp, _dp, _dp, _dp, _dp, _dp,
                                   C.POINTER(C.c_uint8), C.POINTER(C.c_int64)]
        L.or_set_state.argtypes = [vp, _dp, _dp, _dp, _dp, _dp, _dp,
                                   C.POINTER(C.c_uint8), C.c_int64]
        L.or_counters.argtypes = [vp, C.POINTER(C.c_int64)]
        L.or_wall_reactions.argtypes = [vp, _dp]
        L.or_segment_in_particle.argtypes = [vp, C.c_int32, C.c_double, C.c_double,
                                             C.c_double, C.c_double]
        L.or_wall_segment.argtypes = [C.c_double, C.c_double, _dp, _dp]
        L.or_wall_corner.argtypes = [C.c_double, C.c_double, C.c_double, _dp, _dp, _dp]
        L.or_wall_segment_gap.argtypes = [C.c_double, C.c_double]
        L.or_wall_segment_gap.restype = C.c_double
        _LIBS[key] = L
    return _LIBS[key]


def _ptr(a, t):
    return None if a is None else a.ctypes.data_as(C.POINTER(t))


T_PD, T_SELF, T_NBR, T_WALL, T_BODY = 1, 2, 4, 8, 16
T_ALL = 31


class Oracle:
    """One oracle instance over a workloads.Problem."""

    def __init__(self, prob, contact_mode: int = 1, n_threads: int = 1):
        self.lib = _lib(n_threads > 1)
        self.prob = prob
        f64 = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
        i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
        self._keep = keep = dict(
            x=f64(prob.x), y=f64(prob.y), vol=f64(prob.vol),
            po=i32(prob.particle_offset), pm=i32(prob.particle_material),
            pa=i32(prob.particle_aggregate), lo=i32(prob.loop_offset),
            lvo=i32(prob.loop_vertex_offset), lxy=f64(prob.loop_xy) if len(prob.loop_xy) else np.zeros(1),
            box=f64(prob.box).ravel(), vt=f64(prob.top_wall_speed),
            u0x=f64(prob.u0x), u0y=f64(prob.u0y), v0x=f64(prob.v0x), v0y=f64(prob.v0y))
        mats = (_Material * len(prob.materials))()
        for k, m in enumerate(prob.materials):
            mats[k] = _Material(m.rho, m.bulk_k, m.young_E, m.Gc, m.horizon, m.micro)
        keep["mats"] = mats
        pr = _Problem(prob.n_nodes, prob.n_particles, prob.n_aggregates, len(prob.materials),
                      _ptr(keep["x"], C.c_double), _ptr(keep["y"], C.c_double),
                      _ptr(keep["vol"], C.c_double),
                      _ptr(keep["po"], C.c_int32), _ptr(keep["pm"], C.c_int32),
                      _ptr(keep["pa"], C.c_int32), mats,
                      _ptr(keep["lo"], C.c_int32), _ptr(keep["lvo"], C.c_int32),
                      _ptr(keep["lxy"], C.c_double),
                      _ptr(keep["u0x"], C.c_double), _ptr(keep["u0y"], C.c_double),
                      _ptr(keep["v0x"], C.c_double), _ptr(keep["v0y"], C.c_double),
                      prob.contact_radius, prob.friction_mu, prob.damping_ratio, prob.kn_mode,
                      _ptr(keep["box"], C.c_double), _ptr(keep["vt"], C.c_double),
                      prob.gravity[0], prob.gravity[1], prob.dt, contact_mode, n_threads)
        self._pr = pr
        h = C.c_void_p()
        r = self.lib.or_create(C.byref(pr), C.byref(h))
        self.h = h
        if r != 0:
            msg = self.lib.or_error(h).decode() if h else ""
            raise ValueError(f"oracle setup failed ({r}): {msg}")
        self.N = prob.n_nodes

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.or_destroy(h)
            self.h = None

    # -- queries ----------------------------------------------------------
    def constants(self):
        M = len(self.prob.materials)
        out = np.zeros(4 * M)
        self.lib.or_constants(self.h, _ptr(out, C.c_double))
        out = out.reshape(M, 4)
        return dict(cw=out[:, 0], s0=out[:, 1], Kn=out[:, 2], E=out[:, 3])

    def bonds(self):
        nnz = self.lib.or_n_bonds(self.h)
        row = np.zeros(self.N + 1, dtype=np.int32)
        col = np.zeros(max(nnz, 1), dtype=np.int32)
        self.lib.or_bonds(self.h, _ptr(row, C.c_int32), _ptr(col, C.c_int32))
        return row, col[:nnz]

    def step(self, n: int = 1) -> int:
        return int(self.lib.or_step(self.h, int(n)))

    def forces(self, mask: int = T_ALL):
        fx = np.zeros(self.N)
        fy = np.zeros(self.N)
        self.lib.or_forces(self.h, mask, _ptr(fx, C.c_double), _ptr(fy, C.c_double))
        return fx, fy

    def damage(self):
        phi = np.zeros(self.N)
        nb = C.c_int64()
        self.lib.or_damage(self.h, _ptr(phi, C.c_double), C.byref(nb))
        return phi, nb.value

    def contacts(self):
        n = self.lib.or_contacts(self.h, None, None, 0)
        pi = np.zeros(max(n, 1), dtype=np.int32)
        pj = np.zeros(max(n, 1), dtype=np.int32)
        self.lib.or_contacts(self.h, _ptr(pi, C.c_int32), _ptr(pj, C.c_int32), n)
        return pi[:n], pj[:n]

    def get_state(self):
        N = self.N
        arrs = [np.zeros(N) for _ in range(6)]
        nnz = self.lib.or_n_bonds(self.h)
        brk = np.zeros(max(nnz, 1), dtype=np.uint8)
        st = C.c_int64()
        self.lib.or_get_state(self.h, *[_ptr(a, C.c_double) for a in arrs],
                              _ptr(brk, C.c_uint8), C.byref(st))
        return dict(ux=arrs[0], uy=arrs[1], vx=arrs[2], vy=arrs[3], ax=arrs[4], ay=arrs[5],
                    broken=brk[:nnz], step=st.value)

    def set_state(self, s):
        f = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        arrs = [f(s[k]) for k in ("ux", "uy", "vx", "vy", "ax", "ay")]
        brk = np.ascontiguousarray(s["broken"], dtype=np.uint8) if s.get("broken") is not None else None
        self.lib.or_set_state(self.h, *[_ptr(a, C.c_double) for a in arrs],
                              _ptr(brk, C.c_uint8), int(s["step"]))

    def counters(self):
        out = np.zeros(8, dtype=np.int64)
        self.lib.or_counters(self.h, _ptr(out, C.c_int64))
        return dict(inter=out[0], self_=out[1], stick=out[2], slip=out[3], wall=out[4],
                    coincident=out[5], broken=out[6])

    def wall_reactions(self):
        """[n_aggregates, 4 walls (left, right, floor, top), 2]: force the
        particles exert on each wall at the current state"""
        A = self.prob.n_aggregates
        out = np.zeros(8 * A)
        self.lib.or_wall_reactions(self.h, _ptr(out, C.c_double))
        return out.reshape(A, 4, 2)

    def segment_in_particle(self, p, a, b) -> bool:
        return bool(self.lib.or_segment_in_particle(self.h, p, a[0], a[1], b[0], b[1]))


def wall_segment(Rc: float, d: float):
    lib = _lib(False)
    A, g = C.c_double(), C.c_double()
    lib.or_wall_segment(Rc, d, C.byref(A), C.byref(g))
    return A.value, g.value


def wall_corner(Rc: float, da: float, db: float):
    lib = _lib(False)
    A, ix, iy = C.c_double(), C.c_double(), C.c_double()
    lib.or_wall_corner(Rc, da, db, C.byref(A), C.byref(ix), C.byref(iy))
    return A.value, ix.value, iy.value


def wall_segment_gap(Rc: float, d: float) -> float:
    return float(_lib(False).or_wall_segment_gap(Rc, d))
