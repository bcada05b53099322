"""Thin ctypes binding of libhweno.so (include/hweno.h).

Argument marshalling only: every step of the scheme runs in the library's
HIP kernels.  PyTorch supplies device memory (the workspace and the state
tensors) and the current HIP stream.  If the library is missing the calls
raise; there is no fallback.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, 'libhweno.so')

BC = {'periodic': 0, 'outflow': 1, 'inflow': 2, 'slip': 3, 'noslip': 4}

#: size of the library's static device buffer used by hweno_residual_noalloc
NOALLOC_BYTES = 256 << 20

#: every symbol include/hweno.h declares
EXPORTS = ('hweno_default_options', 'hweno_create', 'hweno_destroy', 'hweno_workspace_bytes',
           'hweno_set_workspace', 'hweno_set_inflow_profile', 'hweno_set_inflow_stages',
           'hweno_rk_step_inflow', 'hweno_set_solid', 'hweno_set_solid_state', 'hweno_set_stream',
           'hweno_record_bytes', 'hweno_set_record', 'hweno_rk_step_record',
           'hweno_rk_step_vjp_recorded', 'hweno_take_mu_bar',
           'hweno_set_state', 'hweno_get_state',
           'hweno_residual', 'hweno_residual_noalloc', 'hweno_rk_step', 'hweno_rk_step_source',
           'hweno_residual_vjp',
           'hweno_rk_step_vjp',
           'hweno_set_timing', 'hweno_get_timing', 'hweno_status_string',
           'hweno_batch_create', 'hweno_batch_set_state', 'hweno_batch_get_state',
           'hweno_batch_run', 'hweno_batch_get_diag', 'hweno_get_tiles', 'hweno_set_tiles',
           'hweno_autotune')

#: kernel classes of hweno_timing ('batch' = a whole hweno_batch_run graph,
#: 'fluxup' = face fluxes fused with the update, tiles flux = 0)
KERNEL_CLASSES = ('ghost', 'recon', 'rbar', 'grad', 'flux', 'update', 'batch', 'fluxup')


class Grid(ctypes.Structure):
    _fields_ = [('dim', ctypes.c_int), ('nx', ctypes.c_int), ('ny', ctypes.c_int),
                ('x0', ctypes.c_double), ('x1', ctypes.c_double),
                ('y0', ctypes.c_double), ('y1', ctypes.c_double)]


class PhysicsC(ctypes.Structure):
    _fields_ = [('gamma', ctypes.c_double), ('Pr', ctypes.c_double), ('mu_ref', ctypes.c_double),
                ('mu_exp', ctypes.c_double), ('T_ref', ctypes.c_double)]


class Bcs(ctypes.Structure):
    _fields_ = [('kind', ctypes.c_int * 4), ('inflow', (ctypes.c_double * 4) * 4)]


class OptionsC(ctypes.Structure):
    _fields_ = [('cfl', ctypes.c_double), ('b_visc', ctypes.c_double),
                ('eps_pp', ctypes.c_double), ('eps_weno', ctypes.c_double),
                ('t_final', ctypes.c_double), ('linear_weights', ctypes.c_int),
                ('max_halvings', ctypes.c_int), ('linear_gradients', ctypes.c_int),
                ('keep_stages', ctypes.c_int), ('gradients', ctypes.c_int)]


class Diag(ctypes.Structure):
    _fields_ = [('t', ctypes.c_double), ('dt', ctypes.c_double), ('alpha_star', ctypes.c_double),
                ('beta_max', ctypes.c_double), ('min_rho', ctypes.c_double),
                ('min_p', ctypes.c_double), ('pp_cells', ctypes.c_ulonglong),
                ('restarts', ctypes.c_int), ('pad', ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != 'pad'}


class TilesC(ctypes.Structure):
    _fields_ = [('recon', ctypes.c_int), ('grad', ctypes.c_int), ('flux', ctypes.c_int),
                ('order', ctypes.c_int), ('xcd', ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Timing(ctypes.Structure):
    _fields_ = [('ms', ctypes.c_double * 8), ('launches', ctypes.c_ulonglong * 8)]


class HwenoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__('%s (status %d)' % (msg, code))
        self.code = code


_lib = None


def lib():
    """Load libhweno.so from the package directory (raises if absent)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError('libhweno.so not built: run paper_2608_10569_amd.build.build()')
        L = ctypes.CDLL(LIB_PATH)
        vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
        L.hweno_default_options.argtypes = [ctypes.POINTER(OptionsC)]
        L.hweno_create.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(PhysicsC),
                                   ctypes.POINTER(Bcs), ctypes.POINTER(OptionsC),
                                   ctypes.POINTER(vp)]
        L.hweno_destroy.argtypes = [vp]
        L.hweno_workspace_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.hweno_set_workspace.argtypes = [vp, vp, ctypes.c_size_t]
        L.hweno_set_stream.argtypes = [vp, vp]
        L.hweno_set_inflow_profile.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int]
        L.hweno_set_inflow_stages.argtypes = [vp, ctypes.c_int, vp, vp, vp, ctypes.c_int]
        L.hweno_rk_step_inflow.argtypes = [vp, ctypes.c_double, ctypes.POINTER(Diag)]
        L.hweno_set_solid.argtypes = [vp, vp, ctypes.c_int]
        L.hweno_set_solid_state.argtypes = [vp, vp, dp]
        L.hweno_record_bytes.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
        L.hweno_set_record.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int]
        L.hweno_rk_step_record.argtypes = [vp, ctypes.c_int, vp, ctypes.c_double, vp]
        L.hweno_rk_step_vjp_recorded.argtypes = [vp, ctypes.c_int, vp, vp, dp]
        L.hweno_take_mu_bar.argtypes = [vp, dp]
        L.hweno_set_state.argtypes = [vp, vp, ctypes.c_double]
        L.hweno_get_state.argtypes = [vp, vp, dp]
        L.hweno_residual.argtypes = [vp, vp, vp, vp, ctypes.POINTER(Diag)]
        L.hweno_residual_noalloc.argtypes = [vp, vp, vp, vp, ctypes.POINTER(Diag)]
        L.hweno_rk_step.argtypes = [vp, ctypes.c_double, ctypes.POINTER(Diag)]
        L.hweno_rk_step_source.argtypes = [vp, ctypes.c_double, vp, vp, vp, ctypes.POINTER(Diag)]
        L.hweno_residual_vjp.argtypes = [vp, vp, vp, vp, vp, dp]
        L.hweno_rk_step_vjp.argtypes = [vp, vp, ctypes.c_double, vp, vp, dp]
        L.hweno_set_timing.argtypes = [vp, ctypes.c_int]
        L.hweno_get_timing.argtypes = [vp, ctypes.POINTER(Timing), ctypes.c_int]
        L.hweno_batch_create.argtypes = [ctypes.c_int, ctypes.POINTER(Grid),
                                         ctypes.POINTER(PhysicsC), ctypes.POINTER(Bcs),
                                         ctypes.POINTER(OptionsC), ctypes.POINTER(vp)]
        L.hweno_batch_set_state.argtypes = [vp, ctypes.c_int, vp, ctypes.c_double]
        L.hweno_batch_get_state.argtypes = [vp, ctypes.c_int, vp, dp]
        L.hweno_batch_run.argtypes = [vp, ctypes.c_int]
        L.hweno_batch_get_diag.argtypes = [vp, ctypes.c_int, ctypes.POINTER(Diag)]
        L.hweno_get_tiles.argtypes = [vp, ctypes.POINTER(TilesC)]
        L.hweno_set_tiles.argtypes = [vp, ctypes.POINTER(TilesC)]
        L.hweno_autotune.argtypes = [vp, ctypes.c_int, ctypes.POINTER(TilesC)]
        L.hweno_status_string.argtypes = [ctypes.c_int]
        L.hweno_status_string.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name != 'hweno_status_string':
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def check(code):
    if code != 0:
        raise HwenoError(code, lib().hweno_status_string(code).decode())


GRADIENTS = {'GR': 0, 'DR': 1}


def default_options(**kw):
    o = OptionsC()
    check(lib().hweno_default_options(ctypes.byref(o)))
    for k, v in kw.items():
        if k == 'gradients' and isinstance(v, str):
            v = GRADIENTS[v]
        setattr(o, k, v)
    return o


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """One grid on the current CUDA/HIP device.

    ``bc`` = kinds for (xlo, xhi[, ylo, yhi]); ``inflow`` = {side: primitive
    state (rho, u, [v,] p)}; ``options`` = keyword overrides of the paper's
    defaults (cfl, b_visc, eps_pp, eps_weno, t_final, linear_weights,
    max_halvings, linear_gradients, keep_stages, gradients: 'GR' (default)
    or 'DR', or 0 / 1).
    """

    def __init__(self, nx, ny=None, extent=(0.0, 1.0, 0.0, 1.0), gamma=1.4, Pr=0.72,
                 mu_ref=0.01, mu_exp=0.0, T_ref=1.0, bc=None, inflow=None, device='cuda',
                 **options):
        import torch
        self.dim = 1 if ny is None else 2
        self.nx, self.ny = nx, (ny or 1)
        self.extent = tuple(float(v) for v in extent)
        self.gamma, self.mu_ref = float(gamma), float(mu_ref)
        self.dx = (self.extent[1] - self.extent[0]) / nx
        self.dy = (self.extent[3] - self.extent[2]) / ny if ny else None
        g = Grid(self.dim, nx, ny or 1, *[float(v) for v in
                                          (list(extent) + [0.0, 1.0])[:4]])
        ph = PhysicsC(gamma, Pr, mu_ref, mu_exp, T_ref)
        b = Bcs()
        kinds = bc or ['periodic'] * (2 * self.dim)
        for s, k in enumerate(kinds):
            b.kind[s] = BC[k] if isinstance(k, str) else int(k)
        for s, st in (inflow or {}).items():
            for q, v in enumerate(st):
                b.inflow[s][q] = float(v)
        o = default_options(**options)
        h = ctypes.c_void_p()
        check(lib().hweno_create(ctypes.byref(g), ctypes.byref(ph), ctypes.byref(b),
                                 ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        nb = ctypes.c_size_t()
        check(lib().hweno_workspace_bytes(h, ctypes.byref(nb)))
        dev = torch.device(device)
        if dev.index is None:
            dev = torch.device(dev.type, torch.cuda.current_device())
        self.device = dev
        self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        check(lib().hweno_set_workspace(h, _ptr(self.workspace), nb.value))
        self.set_stream(torch.cuda.current_stream(self.device).cuda_stream)
        self.state_shape = (3, 4, ny, nx) if self.dim == 2 else (2, 3, nx)
        self.vhat_shape = (8, ny, nx) if self.dim == 2 else (3, nx)
        self.record_slots = 0
        self._rec = None

    def set_stream(self, stream):
        check(lib().hweno_set_stream(self._h, ctypes.c_void_p(stream)))

    def set_inflow_profile(self, side, prim):
        """Inflow state per boundary cell of an inflow side (2D): ``prim`` of
        shape (n, 4) with rows (rho, u, v, p), n = ny for sides 0/1 and nx for
        sides 2/3; None restores the side's constant state."""
        import numpy as np
        if prim is None:
            check(lib().hweno_set_inflow_profile(self._h, int(side), None, 0))
            return
        a = np.ascontiguousarray(prim, dtype=np.float64)
        if a.ndim != 2 or a.shape[1] != 4:
            raise ValueError('inflow profile of shape (n, 4) expected')
        check(lib().hweno_set_inflow_profile(self._h, int(side),
                                             a.ctypes.data_as(ctypes.c_void_p), a.shape[0]))

    def set_inflow_stages(self, side, prim1, prim2, prim3):
        """Inflow profiles of side ``side`` at the three stage times (t, t + dt,
        t + dt/2) of the next rk_step_inflow; each of shape (n, 4), rows
        (rho, u, v, p).  All None clears them."""
        import numpy as np
        if prim1 is None and prim2 is None and prim3 is None:
            check(lib().hweno_set_inflow_stages(self._h, int(side), None, None, None, 0))
            return
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (prim1, prim2, prim3)]
        if any(a.ndim != 2 or a.shape[1] != 4 or a.shape != arrs[0].shape for a in arrs):
            raise ValueError('three inflow profiles of equal shape (n, 4) expected')
        check(lib().hweno_set_inflow_stages(self._h, int(side),
                                            *[a.ctypes.data_as(ctypes.c_void_p) for a in arrs],
                                            arrs[0].shape[0]))

    def set_solid(self, mask, wall='slip'):
        """Solid cells inside the grid (bool array (ny, nx)) with reflective
        ('slip') or adiabatic no-slip ('noslip') walls; None removes the mask."""
        import numpy as np
        if mask is None:
            check(lib().hweno_set_solid(self._h, None, 0))
            return
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        if m.shape != (self.ny, self.nx):
            raise ValueError('mask of shape (ny, nx) expected')
        check(lib().hweno_set_solid(self._h, m.ctypes.data_as(ctypes.c_void_p), BC[wall]))

    def set_solid_state(self, fixed, state=None):
        """Solid cells (bool array (ny, nx), each solid in the mask) that hold
        the primitive state (rho, u, v, p) instead of a mirror image; None
        makes every solid cell a mirror again."""
        import numpy as np
        if fixed is None:
            check(lib().hweno_set_solid_state(self._h, None, None))
            return
        f = np.ascontiguousarray(fixed, dtype=np.uint8)
        if f.shape != (self.ny, self.nx):
            raise ValueError('mask of shape (ny, nx) expected')
        st = (ctypes.c_double * 4)(*[float(v) for v in state])
        check(lib().hweno_set_solid_state(self._h, f.ctypes.data_as(ctypes.c_void_p), st))

    def rk_step_inflow(self, dt):
        """One step of fixed dt with the stage inflow profiles; returns diag."""
        d = Diag()
        check(lib().hweno_rk_step_inflow(self._h, float(dt), ctypes.byref(d)))
        return d.as_dict()

    def _dev(self, U):
        import torch
        if U.device != self.device or U.dtype != torch.float64 or not U.is_contiguous():
            raise ValueError('expected a contiguous float64 tensor on %s' % self.device)
        if tuple(U.shape) != self.state_shape:
            raise ValueError('state shape %s, expected %s' % (tuple(U.shape), self.state_shape))
        return U

    def set_state(self, U, t=0.0):
        check(lib().hweno_set_state(self._h, _ptr(self._dev(U)), float(t)))

    def get_state(self):
        import torch
        U = torch.empty(self.state_shape, dtype=torch.float64, device=self.device)
        t = ctypes.c_double()
        check(lib().hweno_get_state(self._h, _ptr(U), ctypes.byref(t)))
        return U, t.value

    def residual(self, U, diag=True):
        """(R, Vhat, diag dict or None) at the state U."""
        import torch
        self._dev(U)
        R = torch.empty(self.state_shape, dtype=torch.float64, device=self.device)
        V = torch.empty(self.vhat_shape, dtype=torch.float64, device=self.device)
        d = Diag()
        check(lib().hweno_residual(self._h, _ptr(U), _ptr(R), _ptr(V),
                                   ctypes.byref(d) if diag else None))
        return R, V, (d.as_dict() if diag else None)

    def residual_noalloc(self, U, diag=True):
        """hweno_residual_noalloc: the residual with the library's static
        device buffer in place of the workspace (same results)."""
        import torch
        self._dev(U)
        R = torch.empty(self.state_shape, dtype=torch.float64, device=self.device)
        V = torch.empty(self.vhat_shape, dtype=torch.float64, device=self.device)
        d = Diag()
        check(lib().hweno_residual_noalloc(self._h, _ptr(U), _ptr(R), _ptr(V),
                                           ctypes.byref(d) if diag else None))
        return R, V, (d.as_dict() if diag else None)

    def residual_vjp(self, U, Rbar, Vbar=None, want_mu=True):
        """(Ubar, mu_bar): adjoint of the residual (and Vhat) at U."""
        import torch
        self._dev(U)
        self._dev(Rbar)
        if Vbar is not None and (tuple(Vbar.shape) != self.vhat_shape or not Vbar.is_contiguous()
                                 or Vbar.dtype != torch.float64):
            raise ValueError('Vbar shape %s, expected %s' % (tuple(Vbar.shape), self.vhat_shape))
        Ub = torch.empty(self.state_shape, dtype=torch.float64, device=self.device)
        mu = ctypes.c_double(0.0)
        check(lib().hweno_residual_vjp(self._h, _ptr(U), _ptr(Rbar),
                                       _ptr(Vbar) if Vbar is not None else None, _ptr(Ub),
                                       ctypes.byref(mu) if want_mu else None))
        return Ub, (mu.value if want_mu else None)

    def rk_step_source(self, dt, src1, src2, src3):
        """One RK3 step of size dt with source moments (layout of R) at t, t+dt, t+dt/2."""
        for q in (src1, src2, src3):
            self._dev(q)
        d = Diag()
        check(lib().hweno_rk_step_source(self._h, float(dt), _ptr(src1), _ptr(src2), _ptr(src3),
                                         ctypes.byref(d)))
        return d.as_dict()

    def rk_step_vjp(self, U0, dt, U3bar, want_mu=True):
        """(U0bar, mu_bar): adjoint of one RK3 step of size dt (held fixed) from U0."""
        import torch
        self._dev(U0)
        self._dev(U3bar)
        U0b = torch.empty(self.state_shape, dtype=torch.float64, device=self.device)
        mu = ctypes.c_double(0.0)
        check(lib().hweno_rk_step_vjp(self._h, _ptr(U0), float(dt), _ptr(U3bar), _ptr(U0b),
                                      ctypes.byref(mu) if want_mu else None))
        return U0b, (mu.value if want_mu else None)

    def set_record(self, nslots):
        """Device buffer for ``nslots`` recorded steps (0 frees it)."""
        import torch
        self._rec = None
        check(lib().hweno_set_record(self._h, None, 0, 0))
        self.record_slots = 0
        if nslots <= 0:
            return
        n = ctypes.c_size_t()
        check(lib().hweno_record_bytes(self._h, int(nslots), ctypes.byref(n)))
        self._rec = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        check(lib().hweno_set_record(self._h, _ptr(self._rec), n.value, int(nslots)))
        self.record_slots = int(nslots)

    def rk_step_record(self, slot, U0, dt):
        """U3 of one fixed step dt from U0, recorded in ``slot`` for
        rk_step_vjp_recorded (the context state is left alone)."""
        import torch
        self._dev(U0)
        U3 = torch.empty(self.state_shape, dtype=torch.float64, device=self.device)
        check(lib().hweno_rk_step_record(self._h, int(slot), _ptr(U0), float(dt), _ptr(U3)))
        return U3

    def take_mu_bar(self):
        """Running sum of the mu adjoints of rk_step_vjp_recorded calls made
        with want_mu=False (cleared by the call)."""
        mu = ctypes.c_double(0.0)
        check(lib().hweno_take_mu_bar(self._h, ctypes.byref(mu)))
        return mu.value

    def rk_step_vjp_recorded(self, slot, U3bar, want_mu=True):
        """(U0bar, mu_bar) of the step recorded in ``slot``; with
        want_mu=False this step's mu adjoint joins the device-side sum that
        take_mu_bar returns (no synchronisation)."""
        import torch
        self._dev(U3bar)
        U0b = torch.empty(self.state_shape, dtype=torch.float64, device=self.device)
        mu = ctypes.c_double(0.0)
        check(lib().hweno_rk_step_vjp_recorded(self._h, int(slot), _ptr(U3bar), _ptr(U0b),
                                               ctypes.byref(mu) if want_mu else None))
        return U0b, (mu.value if want_mu else None)

    def rk_step(self, dt=0.0):
        """One SSP-RK3 step (dt <= 0: the paper's time-step rule); diag dict."""
        d = Diag()
        check(lib().hweno_rk_step(self._h, float(dt), ctypes.byref(d)))
        return d.as_dict()

    def set_timing(self, on=True, classes=None):
        """Record HIP events around the launches of the given kernel classes
        (names of KERNEL_CLASSES; all of them by default) until switched off."""
        mask = 0
        if on:
            names = KERNEL_CLASSES if classes is None else classes
            for nm in names:
                mask |= 1 << KERNEL_CLASSES.index(nm)
        check(lib().hweno_set_timing(self._h, mask))

    def tiles(self):
        t = TilesC()
        check(lib().hweno_get_tiles(self._h, ctypes.byref(t)))
        return t.as_dict()

    def set_tiles(self, recon=32, grad=64, flux=0, order=0, xcd=1):
        t = TilesC(recon, grad, flux, order, xcd)
        check(lib().hweno_set_tiles(self._h, ctypes.byref(t)))

    def autotune(self, reps=3):
        """Times the candidate tiles on the current state(s), keeps the fastest."""
        t = TilesC()
        check(lib().hweno_autotune(self._h, int(reps), ctypes.byref(t)))
        return t.as_dict()

    def timing(self, reset=False):
        """{kernel class: (total ms, launches)} from the library's HIP events."""
        t = Timing()
        check(lib().hweno_get_timing(self._h, ctypes.byref(t), int(bool(reset))))
        return {name: (t.ms[k], t.launches[k]) for k, name in enumerate(KERNEL_CLASSES)}

    def close(self):
        if getattr(self, '_h', None):
            lib().hweno_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch(Solver):
    """Many independent 2D grids advanced together (hweno_batch_*).

    ``problems`` is a list of dicts with the keyword arguments of Solver
    (nx, ny, extent, gamma, Pr, mu_ref, mu_exp, T_ref, bc, inflow and option
    overrides) for each instance.
    """

    def __init__(self, problems, device='cuda'):
        import torch
        n = len(problems)
        grids, phys, bcs, opts = (Grid * n)(), (PhysicsC * n)(), (Bcs * n)(), (OptionsC * n)()
        self.shapes = []
        self.problems = [dict(p) for p in problems]
        for k, pr in enumerate(self.problems):
            pr = dict(pr)
            nx, ny = pr.pop('nx'), pr.pop('ny')
            extent = pr.pop('extent', (0.0, 1.0, 0.0, 1.0))
            grids[k] = Grid(2, nx, ny, *[float(v) for v in extent])
            phys[k] = PhysicsC(pr.pop('gamma', 1.4), pr.pop('Pr', 0.72), pr.pop('mu_ref', 0.01),
                               pr.pop('mu_exp', 0.0), pr.pop('T_ref', 1.0))
            kinds = pr.pop('bc', None) or ['periodic'] * 4
            for s_, kd in enumerate(kinds):
                bcs[k].kind[s_] = BC[kd] if isinstance(kd, str) else int(kd)
            for s_, st in (pr.pop('inflow', None) or {}).items():
                for q, v in enumerate(st):
                    bcs[k].inflow[s_][q] = float(v)
            opts[k] = default_options(**pr)
            self.shapes.append((3, 4, ny, nx))
        h = ctypes.c_void_p()
        check(lib().hweno_batch_create(n, grids, phys, bcs, opts, ctypes.byref(h)))
        self._h = h
        self.n = n
        nb = ctypes.c_size_t()
        check(lib().hweno_workspace_bytes(h, ctypes.byref(nb)))
        dev = torch.device(device)
        if dev.index is None:
            dev = torch.device(dev.type, torch.cuda.current_device())
        self.device = dev
        self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        check(lib().hweno_set_workspace(h, _ptr(self.workspace), nb.value))
        self.set_stream(torch.cuda.current_stream(self.device).cuda_stream)

    def _chk(self, i, U):
        import torch
        if U.device != self.device or U.dtype != torch.float64 or not U.is_contiguous():
            raise ValueError('expected a contiguous float64 tensor on %s' % self.device)
        if tuple(U.shape) != self.shapes[i]:
            raise ValueError('instance %d: shape %s, expected %s' % (i, tuple(U.shape), self.shapes[i]))
        return U

    def set_state(self, i, U, t=0.0):
        check(lib().hweno_batch_set_state(self._h, int(i), _ptr(self._chk(i, U)), float(t)))

    def get_state(self, i):
        import torch
        U = torch.empty(self.shapes[i], dtype=torch.float64, device=self.device)
        t = ctypes.c_double()
        check(lib().hweno_batch_get_state(self._h, int(i), _ptr(U), ctypes.byref(t)))
        return U, t.value

    def run(self, nsteps):
        check(lib().hweno_batch_run(self._h, int(nsteps)))

    def diag(self, i):
        d = Diag()
        check(lib().hweno_batch_get_diag(self._h, int(i), ctypes.byref(d)))
        out = d.as_dict()
        out['steps'] = d.pad
        return out
