"""The oracle: a plain FP64 CPU statement of the batched rigid-body step.

TEST INFRASTRUCTURE ONLY. Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import or run anything in this package.
It shares no code with the HIP library (``paper_2106_13281_amd``): it has its
own parser (``system.py``), its own reset pose and its own C++ stepper
(``orc_step.cpp``, FP64, one environment at a time, templated on the scalar
so that dual numbers give its exact Jacobian and a counting scalar gives the
algorithmic FLOPs of a step).

State layout used here: ``X[env][body][13]`` = p(3), q(4 = w,x,y,z), v(3), w(3).
Actions: ``act[step][env][na]``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from .system import MAXA, MAXB, MAXC, MAXJ, MAXP, System, euler_xyz, mat_to_quat, parse  # noqa: F401

NMARGIN = 8
JUMP_MARGINS = (0, 1, 2)
KINK_MARGINS = (3, 4, 5, 6, 7)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc_step.cpp")
_LIB = os.path.join(_HERE, "liborc.so")


_LIB_NATIVE = os.path.join(_HERE, "liborc_native.so")


def build(force=True):
    """Compile the C++ stepper (plain -O2 for the build machine's baseline
    instruction set, OpenMP over environments): the library the tests load."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + f".tmp{os.getpid()}"
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def use_native():
    """Compile the stepper with -O3 -march=native for the machine this runs on
    and load it in place of the portable build (for timing the oracle on the
    host cores; the source is the same, only the compiler's choices differ,
    e.g. fused multiply-adds). Returns the compile command."""
    global _lib
    tmp = _LIB_NATIVE + f".tmp{os.getpid()}"
    cmd = ["g++", "-O3", "-march=native", "-std=c++17", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_NATIVE)
    _lib = None
    lib(_LIB_NATIVE)
    return " ".join(cmd[:5])


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or 'unknown'."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


class _OrcSys(C.Structure):
    _fields_ = [
        ("nb", C.c_int32), ("nj", C.c_int32), ("nc", C.c_int32), ("na", C.c_int32),
        ("substeps", C.c_int32), ("pad0", C.c_int32),
        ("dt", C.c_double), ("beta", C.c_double), ("elasticity", C.c_double), ("friction", C.c_double),
        ("gravity", C.c_double * 3),
        ("mass", C.c_double * MAXB),
        ("inertia", C.c_double * 3 * MAXB),
        ("free_pos", C.c_double * 3 * MAXB),
        ("free_rot", C.c_double * 3 * MAXB),
        ("c_body", C.c_int32 * MAXC), ("pad1", C.c_int32),
        ("c_local", C.c_double * 3 * MAXC),
        ("c_radius", C.c_double * MAXC),
        ("j_parent", C.c_int32 * MAXJ), ("j_child", C.c_int32 * MAXJ), ("j_dof", C.c_int32 * MAXJ),
        ("pad2", C.c_int32),
        ("j_anchor_p", C.c_double * 3 * MAXJ), ("j_anchor_c", C.c_double * 3 * MAXJ),
        ("j_frame_p", C.c_double * 9 * MAXJ), ("j_frame_c", C.c_double * 9 * MAXJ),
        ("j_k_lin", C.c_double * MAXJ), ("j_c_lin", C.c_double * MAXJ), ("j_k_ang", C.c_double * MAXJ),
        ("j_c_ang", C.c_double * MAXJ), ("j_k_lim", C.c_double * MAXJ),
        ("j_lo", C.c_double * 3 * MAXJ), ("j_hi", C.c_double * 3 * MAXJ),
        ("a_joint", C.c_int32 * MAXA), ("a_axis", C.c_int32 * MAXA),
        ("a_gear", C.c_double * MAXA),
        ("a_mode", C.c_int32 * MAXA),
        ("np", C.c_int32), ("pad3", C.c_int32),
        ("p_a", C.c_int32 * MAXP), ("p_b", C.c_int32 * MAXP), ("p_kind", C.c_int32 * MAXP),
        ("p_a0", C.c_double * 3 * MAXP), ("p_a1", C.c_double * 3 * MAXP), ("p_ra", C.c_double * MAXP),
        ("p_b0", C.c_double * 3 * MAXP), ("p_b1", C.c_double * 3 * MAXP), ("p_rb", C.c_double * MAXP),
        ("p_ah", C.c_double * 3 * MAXP), ("p_bh", C.c_double * 3 * MAXP),
        ("p_aR", C.c_double * 9 * MAXP), ("p_bR", C.c_double * 9 * MAXP),
    ]


_lib = None


def lib(path=None):
    global _lib
    if _lib is None:
        path = path or _LIB
        if path == _LIB and not os.path.exists(_LIB):
            build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        L.orc_sizeof_sys.restype = C.c_int
        L.orc_rollout.argtypes = [C.c_void_p, dp, dp, C.c_int, C.c_int, dp, dp, C.c_int]
        L.orc_rollout.restype = C.c_int
        L.orc_step_jacobian.argtypes = [C.c_void_p, dp, dp, C.c_int, dp, C.c_int]
        L.orc_step_jacobian.restype = C.c_int
        L.orc_count_flops.argtypes = [C.c_void_p, dp, dp]
        L.orc_count_flops.restype = C.c_int64
        L.orc_count_vjp_flops.argtypes = [C.c_void_p, dp, dp]
        L.orc_count_vjp_flops.restype = C.c_int64
        L.orc_quat_to_mat.argtypes = [dp, dp]
        L.orc_joint_angles.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_joint_forces.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.orc_max_threads.restype = C.c_int
        if L.orc_num_margins() != NMARGIN:
            raise RuntimeError("oracle margin count mismatch")
        if L.orc_sizeof_sys() != C.sizeof(_OrcSys):
            raise RuntimeError("oracle struct layout mismatch")
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _pack(flat):
    s = _OrcSys()
    for name, _t in _OrcSys._fields_:
        if name.startswith("pad"):
            continue
        v = flat[name]
        field = getattr(s, name)
        if isinstance(field, (int, float)):
            setattr(s, name, v)
            continue
        arr = np.asarray(v, dtype=np.float64)
        if arr.size == 0:
            continue
        flat_vals = arr.reshape(-1)
        # nested ctypes arrays: fill row by row
        if isinstance(field[0], (int, float)):
            for i, x in enumerate(flat_vals):
                field[i] = type(field[0])(x)
        else:
            inner = len(field[0])
            for i, x in enumerate(flat_vals):
                field[i // inner][i % inner] = x
    return s


class Oracle:
    """FP64 reference for one system description."""

    def __init__(self, text):
        self.system = System(text)
        self._s = _pack(self.system.flat())
        self.nb, self.na, self.nj, self.nc = self.system.nb, self.system.na, self.system.nj, self.system.nc
        self.ns = 13 * self.nb

    @classmethod
    def from_file(cls, path):
        with open(path) as f:
            return cls(f.read())

    # ---------------------------------------------------------------- stepping
    def rollout(self, X, acts, traj=False, margins=False, threads=0):
        """Advance X [E][nb][13] by T = len(acts) steps with acts [T][E][na].

        Returns (X_T, traj [T][E][nb][13] or None, margins [E][7] or None).
        Margins (minimum over the run) are distances to the step's branch
        points: 0 contact depth (m), 1 normal-impulse numerator (m/s),
        2 angle wrap pi - |theta| (rad) — jumps of the result; 3 tangential
        slip speed (m/s), 4 relative Coulomb-cone gap, 5 angle-to-limit
        (rad), 6 action clip gap — kinks of the result.
        """
        X = np.ascontiguousarray(X, dtype=np.float64).copy()
        E = X.shape[0]
        acts = np.ascontiguousarray(acts, dtype=np.float64)
        T = acts.shape[0]
        assert X.shape == (E, self.nb, 13) and acts.shape == (T, E, self.na)
        tr = np.zeros((T, E, self.nb, 13)) if traj else None
        mg = np.zeros((E, NMARGIN)) if margins else None
        rc = lib().orc_rollout(C.byref(self._s), _ptr(X), _ptr(acts) if acts.size else _ptr(np.zeros(1)),
                               E, T, _ptr(tr) if traj else None, _ptr(mg) if margins else None, threads)
        if rc != 0:
            raise RuntimeError("orc_rollout failed")
        return X, tr, mg

    def step(self, X, act, margins=False):
        """One step: X [E][nb][13], act [E][na] -> new X (and margins)."""
        Xn, _, mg = self.rollout(X, np.asarray(act)[None], margins=margins)
        return (Xn, mg) if margins else Xn

    def step_jacobian(self, X, act, threads=0):
        """d(step(X, a))/d(X, a): [E][13nb][13nb + na]."""
        X = np.ascontiguousarray(X, dtype=np.float64)
        act = np.ascontiguousarray(act, dtype=np.float64)
        E = X.shape[0]
        J = np.zeros((E, self.ns, self.ns + self.na))
        a = act if act.size else np.zeros(1)
        rc = lib().orc_step_jacobian(C.byref(self._s), _ptr(X), _ptr(a), E, _ptr(J), threads)
        if rc != 0:
            raise RuntimeError("orc_step_jacobian failed")
        return J

    def step_vjp(self, X, act, g_out):
        """Adjoint of one step: (dL/dX_in [E][nb][13], dL/da [E][na]) for g_out = dL/dX_out."""
        J = self.step_jacobian(X, act)
        E = J.shape[0]
        g = np.einsum("eo,eoi->ei", np.asarray(g_out, dtype=np.float64).reshape(E, self.ns), J)
        return g[:, :self.ns].reshape(E, self.nb, 13), g[:, self.ns:]

    # ---------------------------------------------------------------- parameters
    def param_names(self):
        """System parameters in the library's order: mass per body, principal
        inertia per body (x, y, z), per joint k_lin, c_lin, k_ang, c_ang, k_lim,
        actuator strength per action, friction."""
        names = [("mass", (b,)) for b in range(self.nb)]
        names += [("inertia", (b, k)) for b in range(self.nb) for k in range(3)]
        for f in ("j_k_lin", "j_c_lin", "j_k_ang", "j_c_ang", "j_k_lim"):
            names += [(f, (j,)) for j in range(self.nj)]
        names += [("a_gear", (k,)) for k in range(self.na)]
        names += [("friction", ())]
        return names

    def _param(self, name, idx, value=None):
        field = getattr(self._s, name)
        if not idx:
            if value is not None:
                setattr(self._s, name, value)
            return getattr(self._s, name)
        arr = field if len(idx) == 1 else field[idx[0]]
        if value is not None:
            arr[idx[-1]] = value
        return arr[idx[-1]]

    def param_vjp(self, X, act, g_out, rel=1e-6):
        """g_out . d(step)/d(parameter) for every parameter (param_names order),
        by central differences of the FP64 step with a relative step `rel`
        (absolute for a zero parameter): [E][P]."""
        X = np.asarray(X, dtype=np.float64)
        g = np.asarray(g_out, dtype=np.float64).reshape(len(X), -1)
        out = []
        for name, idx in self.param_names():
            v = float(self._param(name, idx))
            eps = rel * (abs(v) if v != 0.0 else 1.0)
            try:
                self._param(name, idx, v + eps)
                fp = self.step(X, act)
                self._param(name, idx, v - eps)
                fm = self.step(X, act)
            finally:
                self._param(name, idx, v)
            out.append(((fp - fm).reshape(len(X), -1) * g).sum(1) / (2 * eps))
        return np.stack(out, 1)

    def count_flops(self, X, act):
        """Algorithmic floating-point operations of one step of one environment."""
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(self.nb, 13)
        a = np.ascontiguousarray(act, dtype=np.float64).reshape(-1)
        if a.size == 0:
            a = np.zeros(1)
        return int(lib().orc_count_flops(C.byref(self._s), _ptr(X), _ptr(a)))

    def count_vjp_flops(self, X, act):
        """Floating-point operations of one reverse (adjoint) sweep through one
        step of one environment (the forward pass not included)."""
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(self.nb, 13)
        a = np.ascontiguousarray(act, dtype=np.float64).reshape(-1)
        if a.size == 0:
            a = np.zeros(1)
        return int(lib().orc_count_vjp_flops(C.byref(self._s), _ptr(X), _ptr(a)))

    # ---------------------------------------------------------------- pieces
    def joint_angles(self, X):
        """(theta [nj][3], Euler axes [nj][3][3]) of one environment state [nb][13]."""
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(self.nb, 13)
        th = np.zeros((max(self.nj, 1), 3))
        ax = np.zeros((max(self.nj, 1), 3, 3))
        lib().orc_joint_angles(C.byref(self._s), _ptr(X), _ptr(th), _ptr(ax))
        return th[:self.nj], ax[:self.nj]

    def joint_forces(self, X, act=None):
        """Joint + actuator (force, torque) per body [nb][3] at one state (no integration)."""
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(self.nb, 13)
        a = np.zeros(max(self.na, 1)) if act is None else np.ascontiguousarray(act, dtype=np.float64)
        f = np.zeros((self.nb, 3))
        t = np.zeros((self.nb, 3))
        lib().orc_joint_forces(C.byref(self._s), _ptr(X), _ptr(a), _ptr(f), _ptr(t))
        return f, t

    def default_qp(self, angles=None, root_offset=None):
        return self.system.default_qp(angles, root_offset)


def quat_to_mat(q):
    q = np.ascontiguousarray(q, dtype=np.float64)
    R = np.zeros(9)
    lib().orc_quat_to_mat(_ptr(q), _ptr(R))
    return R.reshape(3, 3)


def max_threads():
    return int(lib().orc_max_threads())
