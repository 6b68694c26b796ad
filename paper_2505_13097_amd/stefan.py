"""Python face of the C ABI: one lattice (``Stefan``) on one device.

Argument marshalling only: every step of the method runs in the gfx950
kernels of liblbm_stefan.so.  PyTorch provides the device memory (the
workspace is a uint8 tensor) and the stream (torch's current stream).
"""
import ctypes

import numpy as np
import torch

from . import _lib as C

_BC = {"dirichlet": C.BC_DIRICHLET, "bounceback": C.BC_BOUNCEBACK,
       "periodic": C.BC_PERIODIC, "neumann": C.BC_NEUMANN}
_STORE = {"f64": C.STORE_F64, "f32": C.STORE_F32}
_NEWTON = {"safeguarded": C.NEWTON_SAFEGUARDED, "plain": C.NEWTON_PLAIN}
_SCHEME = {"irebm": C.SCHEME_IREBM, "eebm": C.SCHEME_EEBM,
           "ilfbm": C.SCHEME_ILFBM}
_FRONT = {"integral": C.FRONT_LIQUID_INTEGRAL,
          "crossing": C.FRONT_ZERO_CROSSING}


def make_params(prob, variant=-1, flags=0, strict=False):
    """lbm_stefan_params from a problem description (synth.Problem or an
    object with the same attributes).  Returns (params, keepalive)."""
    p = C.Params()
    p.dim, p.q = prob.dim, prob.q
    p.nx, p.ny = prob.nx, prob.ny
    p.storage = _STORE[prob.storage] if isinstance(prob.storage, str) else prob.storage
    nm = prob.newton_mode
    p.newton_mode = _NEWTON[nm] if isinstance(nm, str) else nm
    p.tau, p.ste, p.t_m, p.delta = prob.tau, prob.ste, prob.tm, prob.delta
    keep = []
    for k in range(4):
        b = prob.bc[k]
        p.bc[k] = _BC[b] if isinstance(b, str) else int(b)
        p.wall_T[k] = prob.wall_T[k]
        prof = prob.wall_profile[k] if prob.wall_profile else None
        if prof is not None:
            arr = np.ascontiguousarray(prof, dtype=np.float64)
            keep.append(arr)
            p.wall_profile[k] = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p.dx = prob.dx or 0.0
    p.newton_tol = prob.tol
    p.newton_max_it = prob.max_it
    p.strict = 1 if strict else 0
    p.variant = variant
    p.flags = flags
    sc = getattr(prob, "scheme", "irebm")
    p.scheme = _SCHEME[sc] if isinstance(sc, str) else int(sc)
    if prob.dim == 3:
        p.nz = prob.nz
        for k in range(2):
            b = prob.bc_z[k]
            p.bc_z[k] = _BC[b] if isinstance(b, str) else int(b)
            p.wall_T_z[k] = prob.wall_T_z[k]
    return p, keep


def _field_shape(prob):
    """(ny, nx), or (nz, ny, nx) on a 3D lattice"""
    if prob.dim == 3:
        return (prob.nz, prob.ny, prob.nx)
    return (prob.ny, prob.nx)


def workspace_bytes(prob, variant=-1, flags=0):
    p, _ = make_params(prob, variant, flags)
    n = ctypes.c_size_t()
    C.check(C.lib().lbm_stefan_workspace_bytes(ctypes.byref(p), ctypes.byref(n)))
    return n.value


def variant_names(q, storage="f32"):
    L = C.lib()
    s = _STORE[storage]
    n = ctypes.c_int32()
    C.check(L.lbm_stefan_variant_count(q, s, ctypes.byref(n)))
    return [L.lbm_stefan_variant_name(q, s, v).decode() for v in range(n.value)]


def step_noalloc(prob, src, dst, stats=False, variant=-1, strict=False,
                 stream=None):
    """One step of prob's lattice from the device state src to dst
    (torch tensors of the state's bytes on the current device) through
    lbm_stefan_step_noalloc: no workspace, nothing allocated.  With
    stats=True waits and returns the step's statistics as a dict."""
    p, keep = make_params(prob, variant, 0, strict)
    st = C.Stats() if stats else None
    s = torch.cuda.current_stream() if stream is None else stream
    rc = C.lib().lbm_stefan_step_noalloc(
        ctypes.byref(p), ctypes.c_void_p(src.data_ptr()),
        ctypes.c_void_p(dst.data_ptr()),
        ctypes.byref(st) if st is not None else None,
        ctypes.c_void_p(s.cuda_stream))
    del keep
    C.check(rc)
    return st.as_dict() if st is not None else None


class Stefan:
    """One lattice on the current CUDA (HIP) device: D1Q3, D2Q5, D2Q9,
    D3Q7 or D3Q19, stepped by IREBM (Algorithm 3), EEBM (Algorithm 2) or
    ILFBM (Algorithm 1, 1D and 2D) as prob.scheme says.

    prob      synth.Problem-like description (lattice, sizes, tau, Ste,
              delta, walls, Newton settings, storage, scheme, initial T0;
              nz and the z walls on a 3D lattice).
    variant   kernel variant (-1: library default).

    Fields come back as (ny, nx) arrays, (nz, ny, nx) in 3D; fronts as
    one value per x row.
    """

    def __init__(self, prob, variant=-1, flags=0, strict=False,
                 device=None, stream=None):
        self.prob = prob
        self._lib = C.lib()
        self.device = torch.device("cuda", torch.cuda.current_device()
                                   if device is None else device)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream() if stream is None else stream
            p, keep = make_params(prob, variant, flags, strict)
            self._params = p
            n = ctypes.c_size_t()
            C.check(self._lib.lbm_stefan_workspace_bytes(ctypes.byref(p),
                                                         ctypes.byref(n)))
            self.workspace = torch.empty(n.value, dtype=torch.uint8,
                                         device=self.device)
            T0 = None
            T0p = None
            if prob.T0 is not None:
                T0 = np.ascontiguousarray(
                    np.broadcast_to(prob.T0, _field_shape(prob)),
                    dtype=np.float64)
                T0p = T0.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            h = ctypes.c_void_p()
            C.check(self._lib.lbm_stefan_init(
                ctypes.byref(p), T0p, ctypes.c_void_p(self.workspace.data_ptr()),
                n.value, ctypes.c_void_p(self.stream.cuda_stream),
                ctypes.byref(h)))
            del keep, T0
        self.h = h
        self.state_dtype = np.float64 if prob.storage == "f64" else np.float32

    # -- time stepping -------------------------------------------------
    def step(self, nsteps, stats=False):
        """Advance nsteps.  With stats=True waits and returns a dict
        (Newton counters, energy, boundary fluxes)."""
        st = C.Stats() if stats else None
        rc = self._lib.lbm_stefan_step(self.h, int(nsteps),
                                       ctypes.byref(st) if st is not None else None)
        C.check(rc, self.h)
        return st.as_dict() if st is not None else None

    def stats(self):
        return self.step(0, stats=True)

    def reset_stats(self):
        C.check(self._lib.lbm_stefan_reset_stats(self.h), self.h)

    # -- queries -------------------------------------------------------
    def front(self, mode="integral"):
        """Front of every row along x: shape (ny,), (nz, ny) in 3D."""
        out = np.empty(_field_shape(self.prob)[:-1])
        C.check(self._lib.lbm_stefan_query_front(
            self.h, _FRONT[mode], out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            None), self.h)
        return out

    def energy(self):
        e = ctypes.c_double()
        C.check(self._lib.lbm_stefan_query_front(
            self.h, C.FRONT_LIQUID_INTEGRAL, None, ctypes.byref(e)), self.h)
        return e.value

    def temperature(self):
        T = np.empty(_field_shape(self.prob))
        C.check(self._lib.lbm_stefan_get_field(
            self.h, C.FIELD_T, ctypes.c_void_p(T.ctypes.data)), self.h)
        return T

    def liquid(self):
        """Liquid fraction of every node (the scheme's own definition)."""
        L = np.empty(_field_shape(self.prob))
        C.check(self._lib.lbm_stefan_get_field(
            self.h, C.FIELD_LIQUID, ctypes.c_void_p(L.ctypes.data)), self.h)
        return L

    def state(self):
        s = np.empty((self.prob.q,) + _field_shape(self.prob),
                     dtype=self.state_dtype)
        C.check(self._lib.lbm_stefan_get_field(
            self.h, C.FIELD_STATE, ctypes.c_void_p(s.ctypes.data)), self.h)
        return s

    def state_ptr(self):
        p = ctypes.c_void_p()
        C.check(self._lib.lbm_stefan_state_ptr(self.h, ctypes.byref(p)), self.h)
        return p.value

    def set_state(self, state):
        """state: host numpy array or device tensor of shape (q, ny, nx)
        ((q, nz, ny, nx) in 3D) and the storage dtype."""
        if isinstance(state, torch.Tensor):
            t = state.contiguous()
            C.check(self._lib.lbm_stefan_set_state(
                self.h, ctypes.c_void_p(t.data_ptr()), 1), self.h)
        else:
            a = np.ascontiguousarray(state, dtype=self.state_dtype)
            C.check(self._lib.lbm_stefan_set_state(
                self.h, ctypes.c_void_p(a.ctypes.data), 0), self.h)

    def set_variant(self, v):
        C.check(self._lib.lbm_stefan_set_variant(self.h, int(v)), self.h)

    def autotune(self, steps=10):
        """Time every kernel variant on this lattice and keep the fastest;
        the state is saved and restored.  Returns (variant, ms per step)."""
        nbytes = self.prob.q * self.prob.nodes * (8 if self.prob.storage == "f64" else 4)
        scratch = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        v = ctypes.c_int32()
        ms = ctypes.c_double()
        C.check(self._lib.lbm_stefan_autotune(
            self.h, ctypes.c_void_p(scratch.data_ptr()), nbytes, int(steps),
            ctypes.byref(v), ctypes.byref(ms)), self.h)
        del scratch
        return v.value, ms.value

    # -- reverse mode (handle created with flags=FLAG_ADJOINT) -----------
    def adjoint_buffers(self):
        a = ctypes.c_void_p()
        b = ctypes.c_void_p()
        C.check(self._lib.lbm_stefan_adjoint_buffers(self.h, ctypes.byref(a),
                                                     ctypes.byref(b)), self.h)
        return a.value, b.value

    def adjoint_reset(self):
        C.check(self._lib.lbm_stefan_adjoint_reset(self.h), self.h)

    def front_vjp(self, state_ptr, dL_dfront, abar_ptr):
        g = np.ascontiguousarray(dL_dfront, dtype=np.float64)
        C.check(self._lib.lbm_stefan_front_vjp(
            self.h, ctypes.c_void_p(state_ptr),
            g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            ctypes.c_void_p(abar_ptr)), self.h)

    def adjoint_step(self, state_ptr, abar_in_ptr, abar_out_ptr):
        C.check(self._lib.lbm_stefan_adjoint_step(
            self.h, ctypes.c_void_p(state_ptr), ctypes.c_void_p(abar_in_ptr),
            ctypes.c_void_p(abar_out_ptr)), self.h)

    def adjoint_initial_state(self, abar_ptr):
        C.check(self._lib.lbm_stefan_adjoint_initial_state(
            self.h, ctypes.c_void_p(abar_ptr)), self.h)

    def adjoint_gradients(self):
        """Returns ({'x-','x+','y-','y+'}: wall gradients, dL/dSte,
        dL/ddelta)."""
        pr = self.prob
        gw = np.zeros(2 * pr.ny + 2 * pr.nx)
        gs = ctypes.c_double()
        gd = ctypes.c_double()
        C.check(self._lib.lbm_stefan_adjoint_gradients(
            self.h, gw.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            ctypes.byref(gs), ctypes.byref(gd)), self.h)
        walls = {"x-": gw[:pr.ny], "x+": gw[pr.ny:2 * pr.ny],
                 "y-": gw[2 * pr.ny:2 * pr.ny + pr.nx],
                 "y+": gw[2 * pr.ny + pr.nx:]}
        return walls, gs.value, gd.value

    def forward_tape(self, nsteps, interval):
        """Advance nsteps storing checkpoints every `interval` steps;
        returns the tape (a device tensor) for backward_tape."""
        n = ctypes.c_size_t()
        C.check(self._lib.lbm_stefan_tape_bytes(ctypes.byref(self._params),
                                                int(nsteps), int(interval),
                                                ctypes.byref(n)))
        tape = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        C.check(self._lib.lbm_stefan_forward_tape(
            self.h, int(nsteps), int(interval), ctypes.c_void_p(tape.data_ptr()),
            n.value), self.h)
        return tape

    def backward_tape(self, dL_dfront, tape):
        """Gradients of a loss with dL/d(final integral front) = dL_dfront
        with respect to the wall temperatures, Ste and delta."""
        pr = self.prob
        g = np.ascontiguousarray(dL_dfront, dtype=np.float64)
        gw = np.zeros(2 * pr.ny + 2 * pr.nx)
        gs = ctypes.c_double()
        gd = ctypes.c_double()
        dp = ctypes.POINTER(ctypes.c_double)
        C.check(self._lib.lbm_stefan_backward_tape(
            self.h, g.ctypes.data_as(dp), ctypes.c_void_p(tape.data_ptr()),
            tape.numel(), gw.ctypes.data_as(dp), ctypes.byref(gs),
            ctypes.byref(gd)), self.h)
        walls = {"x-": gw[:pr.ny], "x+": gw[pr.ny:2 * pr.ny],
                 "y-": gw[2 * pr.ny:2 * pr.ny + pr.nx],
                 "y+": gw[2 * pr.ny + pr.nx:]}
        return walls, gs.value, gd.value

    def close(self):
        if getattr(self, "h", None):
            C.check(self._lib.lbm_stefan_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class StefanBatch:
    """Many independent IREBM lattices (uneven sizes and parameters, one
    lattice type and storage) advanced by one persistent kernel launch per
    step, optionally replayed from a captured hipGraph."""

    def __init__(self, probs, stream=None):
        self.probs = list(probs)
        self._lib = C.lib()
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = torch.cuda.current_stream() if stream is None else stream
        n = len(self.probs)
        arr = (C.Params * n)()
        keep = []
        for k, pr in enumerate(self.probs):
            p, kk = make_params(pr)
            arr[k] = p
            keep.append(kk)
        self._params = arr
        nb = ctypes.c_size_t()
        C.check_batch(self._lib.lbm_stefan_batch_workspace_bytes(arr, n, ctypes.byref(nb)))
        self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        T0s = []
        T0p = (C._c_double_p * n)()
        for k, pr in enumerate(self.probs):
            if pr.T0 is not None:
                a = np.ascontiguousarray(np.broadcast_to(pr.T0, (pr.ny, pr.nx)),
                                         dtype=np.float64)
                T0s.append(a)
                T0p[k] = a.ctypes.data_as(C._c_double_p)
        h = ctypes.c_void_p()
        C.check_batch(self._lib.lbm_stefan_batch_init(
            arr, n, T0p, ctypes.c_void_p(self.workspace.data_ptr()), nb.value,
            ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        del keep, T0s
        self.h = h

    def __len__(self):
        return len(self.probs)

    def set_schedule(self, variant=-1, blocks_per_cu=0, graph_steps=0):
        C.check_batch(self._lib.lbm_stefan_batch_set_schedule(
            self.h, int(variant), int(blocks_per_cu), int(graph_steps)), self.h)

    def step(self, nsteps):
        C.check_batch(self._lib.lbm_stefan_batch_step(self.h, int(nsteps)), self.h)

    def stats(self):
        out = (C.Stats * len(self.probs))()
        C.check_batch(self._lib.lbm_stefan_batch_stats(self.h, out), self.h)
        return [s.as_dict() for s in out]

    def reset_stats(self):
        C.check_batch(self._lib.lbm_stefan_batch_reset_stats(self.h), self.h)

    def front(self, k, mode="integral"):
        out = np.empty(self.probs[k].ny)
        C.check_batch(self._lib.lbm_stefan_batch_query_front(
            self.h, int(k), _FRONT[mode],
            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None), self.h)
        return out

    def energy(self, k):
        e = ctypes.c_double()
        C.check_batch(self._lib.lbm_stefan_batch_query_front(
            self.h, int(k), C.FRONT_LIQUID_INTEGRAL, None, ctypes.byref(e)), self.h)
        return e.value

    def temperature(self, k):
        pr = self.probs[k]
        T = np.empty((pr.ny, pr.nx))
        C.check_batch(self._lib.lbm_stefan_batch_get_field(
            self.h, int(k), C.FIELD_T, ctypes.c_void_p(T.ctypes.data)), self.h)
        return T

    def autotune(self, steps=10):
        """Time every (variant, blocks per CU) pair and keep the fastest;
        states are saved and restored.  Returns (variant, bpc, ms/step)."""
        nb = ctypes.c_size_t()
        C.check_batch(self._lib.lbm_stefan_batch_state_bytes(self.h, ctypes.byref(nb)))
        scratch = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        v = ctypes.c_int32()
        bpc = ctypes.c_int32()
        ms = ctypes.c_double()
        C.check_batch(self._lib.lbm_stefan_batch_autotune(
            self.h, ctypes.c_void_p(scratch.data_ptr()), nb.value, int(steps),
            ctypes.byref(v), ctypes.byref(bpc), ctypes.byref(ms)), self.h)
        del scratch
        return v.value, bpc.value, ms.value

    def close(self):
        if getattr(self, "h", None):
            C.check_batch(self._lib.lbm_stefan_batch_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HotWallFront(torch.autograd.Function):
    """Final integral front position xf(y) of an IREBM run as a function of
    the hot-wall (x-) temperature profile, Ste and delta.

    forward(wall, ste, delta, prob, nsteps, interval): builds the lattice
    of `prob` with these three values, runs nsteps on the GPU keeping a
    checkpoint tape (every `interval` steps, sqrt(nsteps) by default) and
    returns xf (ny,) as a float64 CPU tensor.  backward runs the reverse
    sweep of the tape (recomputing each segment, implicit-function theorem
    at every Newton root) and returns dL/dwall, dL/dSte, dL/ddelta.
    """

    @staticmethod
    def forward(ctx, wall, ste, delta, prob, nsteps, interval=None):
        import math
        interval = interval or max(1, int(round(math.sqrt(nsteps))))
        w = wall.detach().to("cpu", torch.float64).numpy()
        p = prob.with_(wall_profile=(w, prob.wall_profile[1],
                                     prob.wall_profile[2], prob.wall_profile[3]),
                       ste=float(ste), delta=float(delta))
        s = Stefan(p, flags=C.FLAG_ADJOINT)
        tape = s.forward_tape(nsteps, interval)
        xf = torch.from_numpy(s.front("integral"))
        ctx.s, ctx.tape = s, tape
        ctx.dtypes = (wall.dtype, wall.device)
        return xf

    @staticmethod
    def backward(ctx, g):
        walls, gs, gd = ctx.s.backward_tape(g.detach().cpu().numpy(), ctx.tape)
        ctx.s.close()
        ctx.tape = None
        dt, dev = ctx.dtypes
        gw = torch.from_numpy(walls["x-"].copy()).to(dev, dt)
        return (gw, torch.tensor(gs, dtype=torch.float64),
                torch.tensor(gd, dtype=torch.float64), None, None, None)
