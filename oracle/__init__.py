"""CPU FP64 oracle of the IREBM step -- TEST INFRASTRUCTURE ONLY.

This package is the plain, slow, obviously correct statement of what the
GPU path computes: the implicit regularized enthalpy lattice Boltzmann
step of Luddens, Lothode and Danaila (arXiv 2505.13097), Algorithm 3
(Section 4.1), with the boundary closures of Section 4.2, the Neumann
similarity solution of Section 2 and a reverse mode of the step; and the
explicit enthalpy based method the paper compares with (Algorithm 2),
selected by ``prob.scheme == "eebm"``; and both on the 3D lattices D3Q7 and
D3Q19 (``prob.dim == 3``).

Only the tests, the smoke check and the CPU-baseline leg of the bench may
import it.  It shares no code with the GPU library: the C sources in this
directory are compiled with gcc into ``liboracle.so`` and called through
ctypes below.  The state is the distribution functions f[i][y][x]
(f[i][z][y][x] in 3D).
"""
import contextlib
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCES = ("irebm.c", "irebm_cs.c", "eebm.c", "ilfbm.c", "lattice3d.c")

DIRICHLET, BOUNCEBACK, PERIODIC, NEUMANN = 0, 1, 2, 3
SAFEGUARDED, PLAIN = 0, 1
FRONT_INTEGRAL, FRONT_CROSSING = 0, 1
_BC = {"dirichlet": DIRICHLET, "bounceback": BOUNCEBACK, "periodic": PERIODIC,
       "neumann": NEUMANN}
_NEWTON = {"safeguarded": SAFEGUARDED, "plain": PLAIN}


ALT_LIB_PATH = os.path.join(_HERE, "liboracle_alt.so")


def build():
    """Compile liboracle.so with gcc (plain -O2, single thread), and
    liboracle_alt.so: the same sources with phi rounded another way (see
    alternate_rounding)."""
    srcs = [os.path.join(_HERE, s) for s in SOURCES]
    for path, defs in ((LIB_PATH, []), (ALT_LIB_PATH, ["-DORC_PHI_LOGISTIC"])):
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared"] + \
            defs + ["-o", path + ".tmp"] + srcs + ["-lm"]
        subprocess.run(cmd, check=True)
        os.replace(path + ".tmp", path)


class Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("q", ctypes.c_int),
        ("nx", ctypes.c_long), ("ny", ctypes.c_long),
        ("tau", ctypes.c_double), ("ste", ctypes.c_double),
        ("tm", ctypes.c_double), ("delta", ctypes.c_double),
        ("bc", ctypes.c_int * 4), ("wall_T", ctypes.c_double * 4),
        ("wall_profile", ctypes.POINTER(ctypes.c_double) * 4),
        ("tol", ctypes.c_double), ("max_it", ctypes.c_int),
        ("newton_mode", ctypes.c_int), ("dx", ctypes.c_double),
        ("nz", ctypes.c_long), ("bc_z", ctypes.c_int * 2),
        ("wall_T_z", ctypes.c_double * 2), ("scheme", ctypes.c_int),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("max_it", ctypes.c_int), ("nonconverged", ctypes.c_long),
        ("bisections", ctypes.c_long), ("max_residual", ctypes.c_double),
        ("flux_in", ctypes.c_double), ("flux_out", ctypes.c_double),
        ("it_hist", ctypes.c_long * 33),
    ]

    def as_dict(self):
        return {
            "max_it": self.max_it, "nonconverged": self.nonconverged,
            "bisections": self.bisections, "max_residual": self.max_residual,
            "flux_in": self.flux_in, "flux_out": self.flux_out,
            "it_hist": list(self.it_hist),
        }


_lib_handle = None
_alt_handle = None
_use_alt = False


@contextlib.contextmanager
def alternate_rounding():
    """Inside the block every oracle call runs liboracle_alt.so: the same
    scheme with tanh(z) evaluated as 2/(1 + exp(-2z)) - 1 (the other way of
    writing phi), so that the spread between the two results measures how
    strongly an input amplifies rounding.  Not thread-safe."""
    global _use_alt
    prev = _use_alt
    _use_alt = True
    try:
        yield
    finally:
        _use_alt = prev


def lib():
    global _lib_handle, _alt_handle
    if _use_alt:
        if _alt_handle is None:
            if not os.path.exists(ALT_LIB_PATH):
                build()
            _alt_handle = _load(ALT_LIB_PATH)
        return _alt_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib_handle = _load(LIB_PATH)
    return _lib_handle


def _load(path):
    """the library at path with the signatures of its entry points"""
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    P = ctypes.POINTER(Params)
    S = ctypes.POINTER(Stats)
    sig = {
        "orc_lattice": [ctypes.c_int, ctypes.c_int, ip, ip, dp, ip],
        "orc_newton": [ctypes.c_double] * 6 + [ctypes.c_int, ctypes.c_int,
                                               dp, ip, ip],
        "orc_init": [P, dp, dp],
        "orc_step": [P, dp, dp, S],
        "orc_run": [P, dp, ctypes.c_long, S, dp, dp],
        "orc_temperature": [P, dp, dp],
        "orc_energy": [P, dp, dp],
        "orc_front": [P, dp, ctypes.c_int, dp],
        "orc_stefan_lambda": [ctypes.c_double, ctypes.c_double, dp],
        "orc_front_loss": [P, dp, ctypes.c_long, dp, dp],
        "orc_front_loss_grad": [P, dp, ctypes.c_long, dp, dp, dp, dp, dp],
        "orc_adjoint_step": [P, dp, dp, dp, dp, dp, dp],
        "orc_cs_step": [P, dp, dp, ctypes.c_double, ctypes.c_double, dp,
                        dp, dp],
        "orc_cs_front_loss": [P, dp, ctypes.c_long, dp, ctypes.c_double,
                              ctypes.c_double, dp, dp, dp],
        "orc_eebm_init": [P, dp, dp],
        "orc_eebm_step": [P, dp, dp, S],
        "orc_eebm_run": [P, dp, ctypes.c_long, S, dp, dp],
        "orc_eebm_temperature": [P, dp, dp],
        "orc_eebm_energy": [P, dp, dp],
        "orc_eebm_front": [P, dp, ctypes.c_int, dp],
        "orc_eebm_collide": [P, dp, dp],
        "orc_ilfbm_init": [P, dp, dp],
        "orc_ilfbm_step": [P, dp, dp, S],
        "orc_ilfbm_run": [P, dp, ctypes.c_long, S, dp, dp],
        "orc_ilfbm_temperature": [P, dp, dp],
        "orc_ilfbm_energy": [P, dp, dp],
        "orc_ilfbm_front": [P, dp, ctypes.c_int, dp],
        "orc_ilfbm_collide": [P, dp, dp],
        "orc_lattice3": [ctypes.c_int, ip, ip, ip, dp, ip],
        "orc3_init": [P, dp, dp],
        "orc3_step": [P, dp, dp, S],
        "orc3_run": [P, dp, ctypes.c_long, S, dp, dp],
        "orc3_temperature": [P, dp, dp],
        "orc3_energy": [P, dp, dp],
        "orc3_front": [P, dp, ctypes.c_int, dp],
        "orc3_collide": [P, dp, dp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    for name in ("orc_phi", "orc_dphi", "orc_eebm_theta"):
        fn = getattr(L, name)
        fn.argtypes = [ctypes.c_double] * 3
        fn.restype = ctypes.c_double
    L.orc_neumann_T.argtypes = [ctypes.c_double] * 4
    L.orc_neumann_T.restype = ctypes.c_double
    return L


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Setup:
    """orc_params built from a problem description (synth.Problem or any
    object with the same attributes); keeps wall profiles alive."""

    def __init__(self, prob):
        p = Params()
        p.dim, p.q = prob.dim, prob.q
        p.nx, p.ny = prob.nx, prob.ny
        p.tau, p.ste, p.tm, p.delta = prob.tau, prob.ste, prob.tm, prob.delta
        self._keep = []
        for k in range(4):
            b = prob.bc[k]
            p.bc[k] = _BC[b] if isinstance(b, str) else int(b)
            p.wall_T[k] = prob.wall_T[k]
            prof = prob.wall_profile[k] if prob.wall_profile else None
            if prof is not None:
                arr = _f64(prof)
                self._keep.append(arr)
                p.wall_profile[k] = _dp(arr)
        p.tol, p.max_it = prob.tol, prob.max_it
        nm = prob.newton_mode
        p.newton_mode = _NEWTON[nm] if isinstance(nm, str) else int(nm)
        p.dx = prob.dx
        scheme = getattr(prob, "scheme", "irebm")
        self.nz = getattr(prob, "nz", 1) if prob.dim == 3 else 1
        p.nz = self.nz
        if prob.dim == 3:
            for k in range(2):
                b = prob.bc_z[k]
                p.bc_z[k] = _BC[b] if isinstance(b, str) else int(b)
                p.wall_T_z[k] = prob.wall_T_z[k]
            p.scheme = {"irebm": 0, "eebm": 1}.get(scheme, -1)
        self.p = p
        self.q, self.nx, self.ny = prob.q, prob.nx, prob.ny
        self.dim = prob.dim
        # the implicit liquid fraction scheme carries l as one more plane
        self.planes = prob.q + (scheme == "ilfbm")

    @property
    def field(self):
        """shape of a node field"""
        if self.dim == 3:
            return (self.nz, self.ny, self.nx)
        return (self.ny, self.nx)

    @property
    def rows(self):
        """number of rows along x (front values)"""
        return self.ny * self.nz

    @property
    def shape(self):
        return (self.planes,) + self.field

    def ref(self):
        return ctypes.byref(self.p)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle: {what} rejected its arguments (rc={rc})")


def lattice(dim, q):
    ex = (ctypes.c_int * q)()
    ey = (ctypes.c_int * q)()
    w = (ctypes.c_double * q)()
    opp = (ctypes.c_int * q)()
    _check(lib().orc_lattice(dim, q, ex, ey, w, opp), "orc_lattice")
    return (np.array(ex[:]), np.array(ey[:]), np.array(w[:]),
            np.array(opp[:]))


def phi(theta, tm, delta):
    return lib().orc_phi(theta, tm, delta)


def dphi(theta, tm, delta):
    return lib().orc_dphi(theta, tm, delta)


def newton(m0, theta, ste, tm, delta, tol=1e-12, max_it=20,
           mode=SAFEGUARDED):
    out = ctypes.c_double()
    it = ctypes.c_int()
    conv = ctypes.c_int()
    _check(lib().orc_newton(m0, theta, ste, tm, delta, tol, max_it, mode,
                            ctypes.byref(out), ctypes.byref(it),
                            ctypes.byref(conv)), "orc_newton")
    return out.value, it.value, bool(conv.value)


def _fn(prob, name):
    """orc_<name>, or orc_<scheme>_<name> for the comparison schemes, or
    orc3_<name> on the 3D lattices (the scheme travels in the params)."""
    if prob.dim == 3:
        return getattr(lib(), "orc3_" + name)
    scheme = getattr(prob, "scheme", "irebm")
    if scheme in ("eebm", "ilfbm"):
        return getattr(lib(), f"orc_{scheme}_" + name)
    return getattr(lib(), "orc_" + name)


def eebm_theta(H, ste, tm):
    """Temperature of enthalpy H in the explicit scheme (Section 3.4)."""
    return lib().orc_eebm_theta(H, ste, tm)


def eebm_collide(prob, f):
    """Post-collision populations of the explicit scheme's state f
    (Algorithm 2 up to streaming)."""
    s = Setup(prob)
    f = _f64(f)
    out = np.empty_like(f)
    _check(lib().orc_eebm_collide(s.ref(), _dp(f), _dp(out)), "eebm_collide")
    return out


def ilfbm_collide(prob, f):
    """Collision without source of the population planes of an ILFBM
    state (f and l): the populations before the inner loop adds its
    source (Algorithm 1)."""
    s = Setup(prob)
    f = _f64(f)
    out = np.empty((prob.q, prob.ny, prob.nx))
    _check(lib().orc_ilfbm_collide(s.ref(), _dp(f), _dp(out)),
           "ilfbm_collide")
    return out


def lattice3(q):
    """D3Q7 / D3Q19 tables: (ex, ey, ez, w, opp)."""
    t = [(ctypes.c_int * q)() for _ in range(3)]
    w = (ctypes.c_double * q)()
    opp = (ctypes.c_int * q)()
    _check(lib().orc_lattice3(q, t[0], t[1], t[2], w, opp), "orc_lattice3")
    return tuple(np.array(a[:]) for a in t) + (np.array(w[:]),
                                                np.array(opp[:]))


def collide(prob, f):
    """Post-collision populations of a 3D state f (the GPU state)."""
    s = Setup(prob)
    f = _f64(f)
    out = np.empty_like(f)
    _check(lib().orc3_collide(s.ref(), _dp(f), _dp(out)), "orc3_collide")
    return out


def init(prob, T0=None):
    s = Setup(prob)
    f = np.zeros(s.shape)
    T0a = None if T0 is None else _f64(np.broadcast_to(T0, s.field))
    _check(_fn(prob, "init")(s.ref(), _dp(T0a), _dp(f)), "init")
    return f


def step(prob, f):
    s = Setup(prob)
    f = _f64(f)
    out = np.empty_like(f)
    st = Stats()
    _check(_fn(prob, "step")(s.ref(), _dp(f), _dp(out), ctypes.byref(st)),
           "step")
    return out, st.as_dict()


def run(prob, f, nsteps, trace=False):
    """Advance nsteps; returns (f, stats[, energy_trace, flux_trace])."""
    s = Setup(prob)
    f = np.array(f, dtype=np.float64, copy=True, order="C")
    st = Stats()
    et = np.empty(nsteps + 1) if trace else None
    ft = np.empty((nsteps, 2)) if trace else None
    _check(_fn(prob, "run")(s.ref(), _dp(f), nsteps, ctypes.byref(st),
                            _dp(et), _dp(ft)), "run")
    if trace:
        return f, st.as_dict(), et, ft
    return f, st.as_dict()


def temperature(prob, f):
    s = Setup(prob)
    T = np.empty(s.field)
    _check(_fn(prob, "temperature")(s.ref(), _dp(_f64(f)), _dp(T)),
           "temperature")
    return T


def energy(prob, f):
    s = Setup(prob)
    E = ctypes.c_double()
    _check(_fn(prob, "energy")(s.ref(), _dp(_f64(f)), ctypes.byref(E)),
           "energy")
    return E.value


def front(prob, f, mode=FRONT_INTEGRAL):
    """Front per row along x: shape (ny,), or (nz, ny) in 3D."""
    s = Setup(prob)
    xf = np.empty(s.rows)
    _check(_fn(prob, "front")(s.ref(), _dp(_f64(f)), mode, _dp(xf)), "front")
    return xf.reshape(s.nz, s.ny) if s.dim == 3 else xf


def stefan_lambda(ste, theta0):
    lam = ctypes.c_double()
    _check(lib().orc_stefan_lambda(ste, theta0, ctypes.byref(lam)),
           "orc_stefan_lambda")
    return lam.value


def neumann_T(x, t, lam, theta0):
    x = np.asarray(x, dtype=np.float64)
    fn = lib().orc_neumann_T
    return np.vectorize(lambda xx: fn(float(xx), t, lam, theta0))(x)


def front_loss(prob, T0, nsteps, target):
    s = Setup(prob)
    T0a = None if T0 is None else _f64(np.broadcast_to(T0, (s.ny, s.nx)))
    L = ctypes.c_double()
    _check(lib().orc_front_loss(s.ref(), _dp(T0a), nsteps,
                                _dp(_f64(target)), ctypes.byref(L)),
           "orc_front_loss")
    return L.value


def front_loss_grad(prob, T0, nsteps, target):
    """Returns (loss, dL/dT_wall (x- wall, per row), dL/dSte, dL/ddelta)."""
    s = Setup(prob)
    T0a = None if T0 is None else _f64(np.broadcast_to(T0, (s.ny, s.nx)))
    L = ctypes.c_double()
    gw = np.zeros(s.ny)
    gs = ctypes.c_double()
    gd = ctypes.c_double()
    _check(lib().orc_front_loss_grad(s.ref(), _dp(T0a), nsteps,
                                     _dp(_f64(target)), ctypes.byref(L),
                                     _dp(gw), ctypes.byref(gs),
                                     ctypes.byref(gd)), "orc_front_loss_grad")
    return L.value, gw, gs.value, gd.value


def adjoint_step(prob, f, gbar):
    """Returns (fbar, dL/dT_wall contribution, dSte, ddelta) of one step."""
    s = Setup(prob)
    fb = np.empty(s.shape)
    gw = np.zeros(s.ny)
    gs = ctypes.c_double(0.0)
    gd = ctypes.c_double(0.0)
    _check(lib().orc_adjoint_step(s.ref(), _dp(_f64(f)), _dp(_f64(gbar)),
                                  _dp(fb), _dp(gw), ctypes.byref(gs),
                                  ctypes.byref(gd)), "orc_adjoint_step")
    return fb, gw, gs.value, gd.value


def cs_step(prob, f, f_im=None, ste_im=0.0, delta_im=0.0, wall_im=None):
    s = Setup(prob)
    ore = np.empty(s.shape)
    oim = np.empty(s.shape)
    _check(lib().orc_cs_step(s.ref(), _dp(_f64(f)),
                             _dp(None if f_im is None else _f64(f_im)),
                             ste_im, delta_im,
                             _dp(None if wall_im is None else _f64(wall_im)),
                             _dp(ore), _dp(oim)), "orc_cs_step")
    return ore, oim


def cs_front_loss(prob, T0, nsteps, target, ste_im=0.0, delta_im=0.0,
                  wall_im=None):
    s = Setup(prob)
    T0a = None if T0 is None else _f64(np.broadcast_to(T0, (s.ny, s.nx)))
    lr = ctypes.c_double()
    li = ctypes.c_double()
    _check(lib().orc_cs_front_loss(
        s.ref(), _dp(T0a), nsteps, _dp(_f64(target)), ste_im, delta_im,
        _dp(None if wall_im is None else _f64(wall_im)), ctypes.byref(lr),
        ctypes.byref(li)), "orc_cs_front_loss")
    return lr.value, li.value
