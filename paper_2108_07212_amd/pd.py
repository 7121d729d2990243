"""Python binding of libpd (include/pd.h): argument marshalling only.

Every computation runs in libpd's HIP kernels.  torch supplies device memory
(outputs with on_device=True) and the stream; it is imported before libpd is
loaded so that both use the same HIP runtime.  There is no CPU fallback: if
libpd.so has not been built, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpd.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "pd.h")

PD_OK, PD_E_INVALID, PD_E_NOMEM, PD_E_DEVICE, PD_E_NONFINITE, PD_E_ESCAPED, PD_E_STATE = range(7)
TERM_PD, TERM_SELF, TERM_NBR, TERM_WALL, TERM_BODY, TERM_ALL = 1, 2, 4, 8, 16, 31
KERNEL_CLASSES = ("keys", "radix_hist", "radix_digit_scan", "radix_scatter", "cells", "force",
                  "build_list", "pass")


class PDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libpd status {status}: {msg}")
        self.status = status


class Material(C.Structure):
    _fields_ = [("rho", C.c_double), ("bulk_k", C.c_double), ("young_E", C.c_double),
                ("Gc", C.c_double), ("horizon", C.c_double), ("micro", C.c_int32)]


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class Problem(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_particles", C.c_int32), ("n_aggregates", C.c_int32),
                ("n_materials", C.c_int32),
                ("x", _dp), ("y", _dp), ("vol", _dp),
                ("particle_offset", _ip), ("particle_material", _ip), ("particle_aggregate", _ip),
                ("materials", C.POINTER(Material)),
                ("loop_offset", _ip), ("loop_vertex_offset", _ip), ("loop_xy", _dp),
                ("u0x", _dp), ("u0y", _dp), ("v0x", _dp), ("v0y", _dp),
                ("contact_radius", C.c_double), ("friction_mu", C.c_double),
                ("damping_ratio", C.c_double), ("kn_mode", C.c_int32),
                ("box", _dp), ("top_wall_speed", _dp),
                ("gravity_x", C.c_double), ("gravity_y", C.c_double), ("dt", C.c_double),
                ("precision", C.c_int32), ("hip_stream", C.c_void_p)]


class Tuning(C.Structure):
    _fields_ = [("block_nodes", C.c_int32), ("cell_factor", C.c_double),
                ("use_lds", C.c_int32), ("use_graph", C.c_int32), ("skin_factor", C.c_double),
                ("lanes_per_node", C.c_int32), ("wall_pass", C.c_int32)]

    def as_dict(self):
        return dict(block_nodes=self.block_nodes, cell_factor=self.cell_factor,
                    use_lds=self.use_lds, use_graph=self.use_graph, skin_factor=self.skin_factor,
                    lanes_per_node=self.lanes_per_node, wall_pass=self.wall_pass)


_lib = None


def header_functions() -> list:
    """Names of the functions include/pd.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pd_[a-z_]+)\s*\(", txt)))


def load_library(path: str = LIB_PATH):
    """dlopen libpd.so after torch (shared HIP runtime).  Raises if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libpd.so not built at {path}: run __graft_entry__.build()")
    import torch  # noqa: F401  -- HIP runtime first
    L = C.CDLL(path)
    vp = C.c_void_p
    L.pd_setup.argtypes = [C.POINTER(Problem), C.POINTER(vp)]
    L.pd_destroy.argtypes = [vp]
    L.pd_destroy.restype = None
    L.pd_last_error.argtypes = [vp]
    L.pd_last_error.restype = C.c_char_p
    L.pd_step.argtypes = [vp, C.c_int64]
    L.pd_forces.argtypes = [vp, C.c_uint32, vp, vp, C.c_int32]
    L.pd_forces_noalloc.argtypes = [vp, C.c_uint32, vp, vp]
    L.pd_damage.argtypes = [vp, vp, C.POINTER(C.c_int64), C.c_int32]
    L.pd_n_bonds.argtypes = [vp]
    L.pd_n_bonds.restype = C.c_int64
    L.pd_bonds.argtypes = [vp, _ip, _ip]
    L.pd_contacts.argtypes = [vp, _ip, _ip, C.c_int64, C.POINTER(C.c_int64)]
    L.pd_get_state.argtypes = [vp] + [_dp] * 6 + [C.POINTER(C.c_uint8), C.POINTER(C.c_int64)]
    L.pd_set_state.argtypes = [vp] + [_dp] * 6 + [C.POINTER(C.c_uint8), C.c_int64]
    L.pd_counters.argtypes = [vp, C.POINTER(C.c_int64)]
    L.pd_set_counting.argtypes = [vp, C.c_int32]
    L.pd_get_tuning.argtypes = [vp, C.POINTER(Tuning)]
    L.pd_set_tuning.argtypes = [vp, C.POINTER(Tuning)]
    L.pd_autotune.argtypes = [vp, C.c_int32, C.POINTER(Tuning)]
    L.pd_time_kernels.argtypes = [vp, C.c_int64, _dp, _ip, C.c_int32]
    L.pd_sizes.argtypes = [vp, C.POINTER(C.c_int64)]
    L.pd_stream_probe.argtypes = [C.c_int32, vp, vp, C.c_int64, C.c_int32, vp, _dp]
    L.pd_observables.argtypes = [vp, _dp]
    L.pd_particle_damage.argtypes = [vp, vp, C.c_int32]
    L.pd_fragments.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                               C.POINTER(C.c_int64), C.c_int32]
    _fp = C.POINTER(C.c_float)
    L.pd_closure_setup.argtypes = [vp, _ip, C.c_double, _dp, C.c_int32, C.c_double]
    L.pd_closure_modes.argtypes = [vp, C.c_int32, _ip, _ip, _dp, _dp, _dp]
    L.pd_closure_set_modes.argtypes = [vp, C.c_int32, _dp, _dp]
    L.pd_closure_load.argtypes = [vp, C.c_int32, _fp, _fp, _fp]
    L.pd_closure_get.argtypes = [vp, C.c_int32, _fp, _fp, _fp]
    L.pd_closure_enable.argtypes = [vp, C.c_int32]
    L.pd_closure_snapshot.argtypes = [vp, vp, vp, C.c_int32]
    L.pd_closure_forward.argtypes = [vp, C.c_int32, vp, vp, C.c_int64, C.c_int32]
    L.pd_closure_grads.argtypes = [vp, C.c_int32, _dp, _dp, C.c_int64, _fp, _dp]
    L.pd_closure_train.argtypes = [vp, C.c_int32, vp, vp, C.c_int64, C.c_int32, C.c_int32,
                                   C.c_double, C.c_uint64, _fp]
    L.pd_closure_check.argtypes = [vp]
    L.pd_closure_stats.argtypes = [vp, _dp]
    L.pd_closure_particles.argtypes = [vp, _ip, _ip, _ip]
    _lib = L
    return L


CLOSURE_MODES = 32
CLOSURE_PARAMS = 82464
CLOSURE_REDUCED = 4  # pd_closure_enable flag: reduced rigid + modal state


def stream_probe(mode: int, src, dst, reps: int = 10, stream=None) -> float:
    """pd_stream_probe over torch device tensors: mean ms per pass of reading
    (mode 0) or copying (mode 1) all of src."""
    import torch
    L = load_library()
    s = torch.cuda.current_stream() if stream is None else stream
    ms = C.c_double()
    st = L.pd_stream_probe(mode, C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
                           src.numel() * src.element_size(), reps, C.c_void_p(s.cuda_stream),
                           C.byref(ms))
    if st != PD_OK:
        raise PDError(st, "pd_stream_probe")
    return ms.value


def _p(a, t):
    return None if a is None else a.ctypes.data_as(C.POINTER(t))


class PD:
    """One libpd context over a workloads.Problem."""

    def __init__(self, prob, stream=None, precision=None):
        import torch
        self.lib = load_library()
        self.prob = prob
        f64 = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
        i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
        k = self._keep = dict(
            x=f64(prob.x), y=f64(prob.y), vol=f64(prob.vol), po=i32(prob.particle_offset),
            pm=i32(prob.particle_material), pa=i32(prob.particle_aggregate),
            lo=i32(prob.loop_offset), lvo=i32(prob.loop_vertex_offset),
            lxy=f64(prob.loop_xy) if len(prob.loop_xy) else np.zeros(1),
            box=f64(prob.box).ravel(), vt=f64(prob.top_wall_speed),
            u0x=f64(prob.u0x), u0y=f64(prob.u0y), v0x=f64(prob.v0x), v0y=f64(prob.v0y))
        mats = (Material * len(prob.materials))()
        for q, m in enumerate(prob.materials):
            mats[q] = Material(m.rho, m.bulk_k, m.young_E, m.Gc, m.horizon, m.micro)
        k["mats"] = mats
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        prec = prob.precision if precision is None else precision
        pr = Problem(prob.n_nodes, prob.n_particles, prob.n_aggregates, len(prob.materials),
                     _p(k["x"], C.c_double), _p(k["y"], C.c_double), _p(k["vol"], C.c_double),
                     _p(k["po"], C.c_int32), _p(k["pm"], C.c_int32), _p(k["pa"], C.c_int32), mats,
                     _p(k["lo"], C.c_int32), _p(k["lvo"], C.c_int32), _p(k["lxy"], C.c_double),
                     _p(k["u0x"], C.c_double), _p(k["u0y"], C.c_double),
                     _p(k["v0x"], C.c_double), _p(k["v0y"], C.c_double),
                     prob.contact_radius, prob.friction_mu, prob.damping_ratio, prob.kn_mode,
                     _p(k["box"], C.c_double), _p(k["vt"], C.c_double),
                     prob.gravity[0], prob.gravity[1], prob.dt, prec,
                     C.c_void_p(stream.cuda_stream))
        self._pr = pr
        h = C.c_void_p()
        st = self.lib.pd_setup(C.byref(pr), C.byref(h))
        self.h = h
        if st != PD_OK:
            self._raise(st)
        self.N = prob.n_nodes

    def _raise(self, st):
        msg = self.lib.pd_last_error(self.h).decode() if self.h else ""
        raise PDError(st, msg)

    def _chk(self, st):
        if st != PD_OK:
            self._raise(st)

    def close(self):
        if getattr(self, "h", None):
            self.lib.pd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the four calls of the problem statement ---------------------------
    def step(self, n: int = 1, check: bool = True) -> int:
        st = self.lib.pd_step(self.h, int(n))
        if check and st not in (PD_OK,):
            self._raise(st)
        return st

    def forces(self, mask: int = TERM_ALL, device: bool = False):
        if device:
            import torch
            fx = torch.empty(self.N, dtype=torch.float64, device="cuda")
            fy = torch.empty(self.N, dtype=torch.float64, device="cuda")
            self._chk(self.lib.pd_forces(self.h, mask, C.c_void_p(fx.data_ptr()),
                                         C.c_void_p(fy.data_ptr()), 1))
            return fx, fy
        fx = np.zeros(self.N)
        fy = np.zeros(self.N)
        self._chk(self.lib.pd_forces(self.h, mask, C.c_void_p(fx.ctypes.data),
                                     C.c_void_p(fy.ctypes.data), 0))
        return fx, fy

    def forces_noalloc(self, fx, fy, mask: int = TERM_ALL):
        """pd_forces_noalloc into caller-owned device tensors fx, fy (float64, n_nodes)."""
        self._chk(self.lib.pd_forces_noalloc(self.h, mask, C.c_void_p(fx.data_ptr()),
                                             C.c_void_p(fy.data_ptr())))
        return fx, fy

    def damage(self):
        phi = np.zeros(self.N)
        nb = C.c_int64()
        self._chk(self.lib.pd_damage(self.h, C.c_void_p(phi.ctypes.data), C.byref(nb), 0))
        return phi, nb.value

    # -- inspection ------------------------------------------------------------
    def bonds(self):
        nnz = self.lib.pd_n_bonds(self.h)
        row = np.zeros(self.N + 1, dtype=np.int32)
        col = np.zeros(max(nnz, 1), dtype=np.int32)
        self._chk(self.lib.pd_bonds(self.h, _p(row, C.c_int32), _p(col, C.c_int32)))
        return row, col[:nnz]

    def contacts(self):
        cnt = C.c_int64()
        self._chk(self.lib.pd_contacts(self.h, None, None, 0, C.byref(cnt)))
        n = cnt.value
        pi = np.zeros(max(n, 1), dtype=np.int32)
        pj = np.zeros(max(n, 1), dtype=np.int32)
        self._chk(self.lib.pd_contacts(self.h, _p(pi, C.c_int32), _p(pj, C.c_int32), n, C.byref(cnt)))
        return pi[:n], pj[:n]

    def get_state(self):
        arrs = [np.zeros(self.N) for _ in range(6)]
        nnz = self.lib.pd_n_bonds(self.h)
        brk = np.zeros(max(nnz, 1), dtype=np.uint8)
        st = C.c_int64()
        self._chk(self.lib.pd_get_state(self.h, *[_p(a, C.c_double) for a in arrs],
                                        _p(brk, C.c_uint8), C.byref(st)))
        return dict(ux=arrs[0], uy=arrs[1], vx=arrs[2], vy=arrs[3], ax=arrs[4], ay=arrs[5],
                    broken=brk[:nnz], step=st.value)

    def set_state(self, s):
        f = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        arrs = [f(s[k]) for k in ("ux", "uy", "vx", "vy", "ax", "ay")]
        brk = None if s.get("broken") is None else np.ascontiguousarray(s["broken"], dtype=np.uint8)
        self._chk(self.lib.pd_set_state(self.h, *[_p(a, C.c_double) for a in arrs],
                                        _p(brk, C.c_uint8), int(s["step"])))

    def counters(self):
        out = np.zeros(8, dtype=np.int64)
        self._chk(self.lib.pd_counters(self.h, _p(out, C.c_int64)))
        return dict(inter=out[0], self_=out[1], stick=out[2], slip=out[3], wall=out[4],
                    coincident=out[5], broken=out[6], steps=out[7])

    def set_counting(self, on: bool = True):
        self._chk(self.lib.pd_set_counting(self.h, 1 if on else 0))

    def tuning(self) -> dict:
        t = Tuning()
        self._chk(self.lib.pd_get_tuning(self.h, C.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        t = Tuning()
        self._chk(self.lib.pd_get_tuning(self.h, C.byref(t)))
        for k, v in kw.items():
            setattr(t, k, v)
        self._chk(self.lib.pd_set_tuning(self.h, C.byref(t)))

    def autotune(self, steps: int = 20) -> dict:
        t = Tuning()
        self._chk(self.lib.pd_autotune(self.h, int(steps), C.byref(t)))
        return t.as_dict()

    def time_kernels(self, n_steps: int = 10):
        """{kernel class: (mean ms per launch, launches over the n_steps steps)}"""
        ms = np.zeros(8)
        la = np.zeros(8, dtype=np.int32)
        self._chk(self.lib.pd_time_kernels(self.h, int(n_steps), _p(ms, C.c_double),
                                           _p(la, C.c_int32), 8))
        return {k: (float(ms[i]), int(la[i])) for i, k in enumerate(KERNEL_CLASSES)}

    def sizes(self) -> dict:
        out = np.zeros(10, dtype=np.int64)
        self._chk(self.lib.pd_sizes(self.h, _p(out, C.c_int64)))
        keys = ("nodes", "bonds", "slots", "cells", "radix_passes", "particles", "aggregates",
                "max_window", "list_rebuilds", "list_slots")
        return {k: int(v) for k, v in zip(keys, out)}

    # -- compaction observables -------------------------------------------
    def observables(self):
        """dict of per-aggregate arrays: wall_force [A, 4, 2] (left, right,
        floor, top; force on the wall), volume_fraction, broken, reference
        (directed bonds), top_wall_y"""
        A = self.prob.n_aggregates
        out = np.zeros(12 * A)
        self._chk(self.lib.pd_observables(self.h, _p(out, C.c_double)))
        o = out.reshape(A, 12)
        return dict(wall_force=o[:, :8].reshape(A, 4, 2), volume_fraction=o[:, 8],
                    broken=o[:, 9], reference=o[:, 10], top_wall_y=o[:, 11])

    def particle_damage(self):
        out = np.zeros(self.prob.n_particles)
        self._chk(self.lib.pd_particle_damage(self.h, C.c_void_p(out.ctypes.data), 0))
        return out

    def fragments(self, min_nodes: int = 1):
        """(label [N] int32: smallest node index of each node's component of
        the intact-bond graph, count [P] int32: components per particle with
        at least min_nodes nodes, number of all components)"""
        lab = np.zeros(self.N, dtype=np.int32)
        cnt = np.zeros(self.prob.n_particles, dtype=np.int32)
        nc = C.c_int64()
        self._chk(self.lib.pd_fragments(self.h, int(min_nodes), _p(lab, C.c_int32),
                                        _p(cnt, C.c_int32), C.byref(nc), 0))
        return lab, cnt, nc.value

    # -- learned modal closure ---------------------------------------------
    def closure_setup(self, shape_of_particle, gate_frac: float = 0.5, tau_c=None,
                      check_every: int = 100, err_tol: float = 0.05):
        sp = np.ascontiguousarray(shape_of_particle, dtype=np.int32)
        tc = None if tau_c is None else np.ascontiguousarray(tau_c, dtype=np.float64)
        self._chk(self.lib.pd_closure_setup(self.h, _p(sp, C.c_int32), float(gate_frac),
                                            _p(tc, C.c_double), int(check_every), float(err_tol)))
        st = self.closure_stats()
        self.n_closure, self.n_shapes = int(st["particles"]), int(st["shapes"])

    def closure_modes(self, shape: int):
        """(phi [n_nodes, 32, 2], lambda [32], sigma [32], mode count)"""
        nn, nm = C.c_int32(), C.c_int32()
        self._chk(self.lib.pd_closure_modes(self.h, shape, C.byref(nn), C.byref(nm), None, None, None))
        phi = np.zeros((nn.value, CLOSURE_MODES, 2))
        lam, sig = np.zeros(CLOSURE_MODES), np.zeros(CLOSURE_MODES)
        self._chk(self.lib.pd_closure_modes(self.h, shape, None, None, _p(phi, C.c_double),
                                            _p(lam, C.c_double), _p(sig, C.c_double)))
        return phi, lam, sig, nm.value

    def closure_set_modes(self, shape: int, phi, lam):
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        self._chk(self.lib.pd_closure_set_modes(self.h, shape, _p(phi, C.c_double),
                                                _p(lam, C.c_double)))

    def closure_load(self, shape: int, params, sig_q=None, sig_r=None):
        f = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float32)
        params, sig_q, sig_r = f(params), f(sig_q), f(sig_r)
        assert params.size == CLOSURE_PARAMS
        self._chk(self.lib.pd_closure_load(self.h, shape, _p(params, C.c_float),
                                           _p(sig_q, C.c_float), _p(sig_r, C.c_float)))

    def closure_get(self, shape: int):
        p = np.zeros(CLOSURE_PARAMS, dtype=np.float32)
        sq = np.zeros(CLOSURE_MODES, dtype=np.float32)
        sr = np.zeros(CLOSURE_MODES, dtype=np.float32)
        self._chk(self.lib.pd_closure_get(self.h, shape, _p(p, C.c_float), _p(sq, C.c_float),
                                          _p(sr, C.c_float)))
        return p, sq, sr

    def closure_enable(self, mode: int):
        self._chk(self.lib.pd_closure_enable(self.h, int(mode)))

    def closure_snapshot(self, device: bool = False):
        """(q, g) [closure particles, 32]: modal amplitudes and modal plain bond force"""
        n = self.n_closure
        if device:
            import torch
            q = torch.empty((n, CLOSURE_MODES), dtype=torch.float64, device="cuda")
            g = torch.empty((n, CLOSURE_MODES), dtype=torch.float64, device="cuda")
            self._chk(self.lib.pd_closure_snapshot(self.h, C.c_void_p(q.data_ptr()),
                                                   C.c_void_p(g.data_ptr()), 1))
            return q, g
        q = np.zeros((n, CLOSURE_MODES))
        g = np.zeros((n, CLOSURE_MODES))
        self._chk(self.lib.pd_closure_snapshot(self.h, C.c_void_p(q.ctypes.data),
                                               C.c_void_p(g.ctypes.data), 0))
        return q, g

    def closure_forward(self, shape: int, q):
        """g = -lambda q + sigma_r MLP(q / sigma_q) (numpy in, numpy out, or
        cuda float64 tensors in and out)"""
        if hasattr(q, "data_ptr"):
            import torch
            q = q.contiguous()
            g = torch.empty_like(q)
            self._chk(self.lib.pd_closure_forward(self.h, shape, C.c_void_p(q.data_ptr()),
                                                  C.c_void_p(g.data_ptr()), q.shape[0], 1))
            return g
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, CLOSURE_MODES)
        g = np.zeros_like(q)
        self._chk(self.lib.pd_closure_forward(self.h, shape, C.c_void_p(q.ctypes.data),
                                              C.c_void_p(g.ctypes.data), q.shape[0], 0))
        return g

    def closure_grads(self, shape: int, q, g):
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, CLOSURE_MODES)
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(-1, CLOSURE_MODES)
        out = np.zeros(CLOSURE_PARAMS, dtype=np.float32)
        loss = C.c_double()
        self._chk(self.lib.pd_closure_grads(self.h, shape, _p(q, C.c_double), _p(g, C.c_double),
                                            q.shape[0], _p(out, C.c_float), C.byref(loss)))
        return loss.value, out

    def closure_train(self, shape: int, q, g, iters: int = 2000, batch: int = 512,
                      lr: float = 1e-3, seed: int = 0):
        """Train on cuda float64 tensors q, g [n, 32]; returns the loss per iteration."""
        q, g = q.contiguous(), g.contiguous()
        loss = np.zeros(iters, dtype=np.float32)
        self._chk(self.lib.pd_closure_train(self.h, shape, C.c_void_p(q.data_ptr()),
                                            C.c_void_p(g.data_ptr()), q.shape[0], int(iters),
                                            int(batch), float(lr), int(seed),
                                            _p(loss, C.c_float)))
        return loss

    def closure_check(self):
        self._chk(self.lib.pd_closure_check(self.h))

    def closure_stats(self) -> dict:
        out = np.zeros(8)
        self._chk(self.lib.pd_closure_stats(self.h, _p(out, C.c_double)))
        keys = ("particles", "active", "fallbacks", "checks", "err", "err_linear", "checked",
                "shapes")
        return dict(zip(keys, out.tolist()))

    def closure_particles(self):
        n = self.n_closure
        p, s, a = (np.zeros(n, dtype=np.int32) for _ in range(3))
        self._chk(self.lib.pd_closure_particles(self.h, _p(p, C.c_int32), _p(s, C.c_int32),
                                                _p(a, C.c_int32)))
        return p, s, a
