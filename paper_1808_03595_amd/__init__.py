"""MI355X p-multigrid solver for the statically condensed SEM Helmholtz problem.

Thin ctypes binding of the C ABI declared in ``include/pmg.h``
(``libpmg.so``, built in-tree by ``paper_1808_03595_amd.build``).  Every
function keeps the name of its C entry point without the ``pmg_`` prefix and
only marshals arguments: device arrays may be passed as torch tensors (their
``data_ptr()`` is used) or as raw integer addresses; streams default to
torch's current stream.  All computation happens in the HIP library; if the
library is missing the import of this package still works but every call
raises ``RuntimeError``.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpmg.so")

F64 = 0
F32 = 1
MAX_HIST = 512
NOT_CONVERGED = 1
BREAKDOWN = 2
EINVAL = -1
EUNSUP = -4

_lib = None


class PmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pmg error {code}: {msg}")
        self.code = code


class Stats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int),
        ("status", ctypes.c_int),
        ("res0", ctypes.c_double),
        ("rel_res", ctypes.c_double),
        ("res_hist", ctypes.c_double * MAX_HIST),
        ("coarse_iters", ctypes.c_int),
        ("t_pre_ms", ctypes.c_double),
        ("t_iter_ms", ctypes.c_double),
        ("t_post_ms", ctypes.c_double),
    ]

    def history(self):
        return [self.res_hist[k] for k in range(min(self.iters + 1, MAX_HIST))]


_VP = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_F = ctypes.c_float
_I64P = ctypes.POINTER(ctypes.c_int64)
_IP = ctypes.POINTER(ctypes.c_int)
_DP = ctypes.POINTER(ctypes.c_double)
_FP = ctypes.POINTER(ctypes.c_float)

# name -> (restype, argtypes)
SIGNATURES = {
    "pmg_create_mesh": (_I, [_I, _I, _I, _I, _D, _D, ctypes.POINTER(_VP)]),
    "pmg_create_mesh_widths": (_I, [_I, _I, _I, _I, _D, _DP, _DP, _DP, ctypes.POINTER(_VP)]),
    "pmg_create_mesh_bc": (_I, [_I, _I, _I, _I, _D, _DP, _DP, _DP, _IP, ctypes.POINTER(_VP)]),
    "pmg_destroy_mesh": (None, [_VP]),
    "pmg_num_levels": (_I, [_VP, _IP]),
    "pmg_level_degree": (_I, [_VP, _I, _IP]),
    "pmg_skeleton_len": (_I, [_VP, _I, _I64P]),
    "pmg_grid_len": (_I, [_VP, _I64P]),
    "pmg_grid_coords": (_I, [_VP, _DP, _DP, _DP]),
    "pmg_grid_to_skeleton": (_I, [_VP, _I, _VP, _VP, _VP]),
    "pmg_skeleton_to_grid": (_I, [_VP, _I, _VP, _VP, _VP]),
    "pmg_apply_condensed_op": (_I, [_VP, _I, _I, _VP, _VP, _VP]),
    "pmg_schwarz_smooth": (_I, [_VP, _I, _I, _VP, _VP, _D, _VP]),
    "pmg_schwarz_smooth_add": (_I, [_VP, _I, _I, _VP, _VP, _D, _VP]),
    "pmg_prolong_add": (_I, [_VP, _I, _I, _VP, _VP, _VP]),
    "pmg_restrict": (_I, [_VP, _I, _I, _VP, _VP, _VP]),
    "pmg_set_cycle": (_I, [_VP, _I, _D, _I]),
    "pmg_set_smoother": (_I, [_VP, _I]),
    "pmg_set_coarse_level": (_I, [_VP, _I]),
    "pmg_set_coarse_solver": (_I, [_VP, _I]),
    "pmg_set_damping": (_I, [_VP, _FP, _I]),
    "pmg_set_coarse_mg": (_I, [_VP, _I, _D, _I]),
    "pmg_vcycle": (_I, [_VP, _I, _VP, _VP, _VP]),
    "pmg_coarse_solve": (_I, [_VP, _VP, _VP, _IP, _VP]),
    "pmg_condense_rhs": (_I, [_VP, _VP, _VP, _VP]),
    "pmg_recover_interior": (_I, [_VP, _VP, _VP, _VP, _VP]),
    "pmg_pcg_solve": (_I, [_VP, _VP, _VP, _D, _I, _I, ctypes.POINTER(Stats), _VP]),
    "pmg_mg_solve": (_I, [_VP, _VP, _VP, _D, _I, ctypes.POINTER(Stats), _VP]),
    "pmg_lift_dirichlet": (_I, [_VP, _VP, _VP, _VP, _VP]),
    "pmg_set_boundary": (_I, [_VP, _VP, _VP, _VP]),
    "pmg_pcg_solve_dirichlet": (_I, [_VP, _VP, _VP, _VP, _D, _I, _I, ctypes.POINTER(Stats), _VP]),
    "pmg_mlp_nparams": (_I, [_I]),
    "pmg_mlp_forward": (_I, [_VP, _VP, _VP, _VP, _I, _I, _VP]),
    "pmg_mlp_loss": (_I, [_VP, _VP, _VP, _VP, _VP, _I, _I, _VP]),
    "pmg_mlp_backward": (_I, [_VP, _VP, _VP, _VP, _VP, _I, _I, _VP]),
    "pmg_mlp_backward_noalloc": (_I, [_VP, _VP, _VP, _VP, _VP, _I, _I, _VP]),
    "pmg_mlp_adam": (_I, [_VP, _VP, _VP, _VP, _I, _F, _F, _F, _F, _I, _VP]),
    "pmg_last_error": (ctypes.c_char_p, []),
}


def lib():
    """Load libpmg.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} not found: build it with python -m paper_1808_03595_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def _check(rc, allow_status=False):
    if rc < 0 or (rc > 0 and not allow_status):
        msg = lib().pmg_last_error().decode()
        raise PmgError(rc, msg)
    return rc


class Mesh:
    """Owning wrapper of a ``pmg_mesh`` handle."""

    def __init__(self, handle, n, p, lam):
        self.h = handle
        self.n = tuple(n)
        self.p = p
        self.lam = lam

    def __del__(self):
        if getattr(self, "h", None):
            try:
                lib().pmg_destroy_mesh(self.h)
            except Exception:
                pass
            self.h = None

    def close(self):
        self.__del__()

    # ---- queries ---------------------------------------------------------
    def num_levels(self):
        L = ctypes.c_int()
        _check(lib().pmg_num_levels(self.h, ctypes.byref(L)))
        return L.value

    def level_degree(self, level):
        p = ctypes.c_int()
        _check(lib().pmg_level_degree(self.h, level, ctypes.byref(p)))
        return p.value

    def skeleton_len(self, level=None):
        if level is None:
            level = self.num_levels()
        n = ctypes.c_int64()
        _check(lib().pmg_skeleton_len(self.h, level, ctypes.byref(n)))
        return n.value

    def grid_len(self):
        n = ctypes.c_int64()
        _check(lib().pmg_grid_len(self.h, ctypes.byref(n)))
        return n.value

    def grid_shape(self):
        N = [self.n[d] * self.p + 1 for d in range(3)]
        return (N[2], N[1], N[0])

    def grid_coords(self):
        N = [self.n[d] * self.p + 1 for d in range(3)]
        arrs = [(ctypes.c_double * N[d])() for d in range(3)]
        _check(lib().pmg_grid_coords(self.h, arrs[0], arrs[1], arrs[2]))
        return [list(a) for a in arrs]

    # ---- operators ---------------------------------------------------------
    def grid_to_skeleton(self, grid, skel, dtype=F64, stream=None):
        _check(lib().pmg_grid_to_skeleton(self.h, dtype, _ptr(grid), _ptr(skel), _stream(stream)))

    def skeleton_to_grid(self, skel, grid, dtype=F64, stream=None):
        _check(lib().pmg_skeleton_to_grid(self.h, dtype, _ptr(skel), _ptr(grid), _stream(stream)))

    def apply_condensed_op(self, level, u, y, dtype=F64, stream=None):
        _check(lib().pmg_apply_condensed_op(self.h, level, dtype, _ptr(u), _ptr(y), _stream(stream)))

    def schwarz_smooth(self, level, r, du, omega=1.0, dtype=F64, stream=None):
        _check(lib().pmg_schwarz_smooth(self.h, level, dtype, _ptr(r), _ptr(du), omega, _stream(stream)))

    def schwarz_smooth_add(self, level, r, u, omega=1.0, dtype=F64, stream=None):
        _check(lib().pmg_schwarz_smooth_add(self.h, level, dtype, _ptr(r), _ptr(u), omega, _stream(stream)))

    def prolong_add(self, level, coarse, fine, dtype=F64, stream=None):
        _check(lib().pmg_prolong_add(self.h, level, dtype, _ptr(coarse), _ptr(fine), _stream(stream)))

    def restrict(self, level, fine, coarse, dtype=F64, stream=None):
        _check(lib().pmg_restrict(self.h, level, dtype, _ptr(fine), _ptr(coarse), _stream(stream)))

    def set_cycle(self, nu_mode=0, coarse_rtol=1e-8, coarse_maxit=2000):
        _check(lib().pmg_set_cycle(self.h, nu_mode, coarse_rtol, coarse_maxit))

    def set_coarse_mg(self, levels=0, omega=0.6, nu=1):
        _check(lib().pmg_set_coarse_mg(self.h, levels, omega, nu))

    def set_coarse_solver(self, kind=0):
        """0: Jacobi CG (Sec. 4.1); 1: exact solve by fast diagonalization."""
        _check(lib().pmg_set_coarse_solver(self.h, kind))

    def set_coarse_level(self, level=0):
        _check(lib().pmg_set_coarse_level(self.h, level))

    def set_smoother(self, kind=0):
        """0: star smoother (Alg. 2); 1: element-centred blocks (Sec. 3.4)."""
        _check(lib().pmg_set_smoother(self.h, kind))

    def set_damping(self, omega=None):
        if omega is None or len(omega) == 0:
            _check(lib().pmg_set_damping(self.h, None, 0))
            return
        arr = (ctypes.c_float * len(omega))(*[float(w) for w in omega])
        _check(lib().pmg_set_damping(self.h, arr, len(omega)))

    def vcycle(self, r, z, dtype=F64, stream=None):
        _check(lib().pmg_vcycle(self.h, dtype, _ptr(r), _ptr(z), _stream(stream)))

    def coarse_solve(self, F0, u0, stream=None):
        it = ctypes.c_int()
        _check(lib().pmg_coarse_solve(self.h, _ptr(F0), _ptr(u0), ctypes.byref(it), _stream(stream)))
        return it.value

    def condense_rhs(self, f, Fhat, stream=None):
        _check(lib().pmg_condense_rhs(self.h, _ptr(f), _ptr(Fhat), _stream(stream)))

    def recover_interior(self, f, uhat, u, stream=None):
        _check(lib().pmg_recover_interior(self.h, _ptr(f), _ptr(uhat), _ptr(u), _stream(stream)))

    def pcg_solve(self, f, u, rtol=1e-10, maxit=200, precond_dtype=F64, stream=None):
        st = Stats()
        _check(lib().pmg_pcg_solve(self.h, _ptr(f), _ptr(u), rtol, maxit, precond_dtype,
                                   ctypes.byref(st), _stream(stream)), allow_status=True)
        return st

    def mg_solve(self, f, u, rtol=1e-10, maxit=200, stream=None):
        st = Stats()
        _check(lib().pmg_mg_solve(self.h, _ptr(f), _ptr(u), rtol, maxit, ctypes.byref(st),
                                  _stream(stream)), allow_status=True)
        return st

    def lift_dirichlet(self, f, g, out, stream=None):
        _check(lib().pmg_lift_dirichlet(self.h, _ptr(f), _ptr(g), _ptr(out), _stream(stream)))

    def set_boundary(self, g, u, stream=None):
        _check(lib().pmg_set_boundary(self.h, _ptr(g), _ptr(u), _stream(stream)))

    def pcg_solve_dirichlet(self, f, g, u, rtol=1e-10, maxit=200, precond_dtype=F64, stream=None):
        st = Stats()
        _check(lib().pmg_pcg_solve_dirichlet(self.h, _ptr(f), _ptr(g), _ptr(u), rtol, maxit,
                                             precond_dtype, ctypes.byref(st), _stream(stream)),
               allow_status=True)
        return st


def create_mesh(n1, n2, n3, p, lam, stretch=1.0):
    h = _VP()
    _check(lib().pmg_create_mesh(n1, n2, n3, p, lam, stretch, ctypes.byref(h)))
    return Mesh(h, (n1, n2, n3), p, lam)


def create_mesh_widths(hx, hy, hz, p, lam):
    arrs = [(ctypes.c_double * len(a))(*[float(v) for v in a]) for a in (hx, hy, hz)]
    h = _VP()
    _check(lib().pmg_create_mesh_widths(len(hx), len(hy), len(hz), p, lam, arrs[0], arrs[1],
                                        arrs[2], ctypes.byref(h)))
    return Mesh(h, (len(hx), len(hy), len(hz)), p, lam)


BC_DIRICHLET, BC_NEUMANN, BC_PERIODIC = 0, 1, 2
_BC_CODE = {"D": BC_DIRICHLET, "N": BC_NEUMANN, "P": BC_PERIODIC}


def bc_codes(bc):
    """Six side kinds (x1 low, x1 high, x2 low, ..., x3 high) from a string
    such as "DNPPDD", or three per-direction entries each "D"/"N"/"P" or a
    (low, high) pair."""
    if isinstance(bc, str) and len(bc) == 6:
        sides = list(bc)
    else:
        sides = []
        for b in bc:
            sides += [b, b] if isinstance(b, str) and len(b) == 1 else [b[0], b[1]]
    return [_BC_CODE[s] if isinstance(s, str) else int(s) for s in sides]


def create_mesh_bc(hx, hy, hz, p, lam, bc):
    arrs = [(ctypes.c_double * len(a))(*[float(v) for v in a]) for a in (hx, hy, hz)]
    codes = (ctypes.c_int * 6)(*bc_codes(bc))
    h = _VP()
    _check(lib().pmg_create_mesh_bc(len(hx), len(hy), len(hz), p, lam, arrs[0], arrs[1], arrs[2], codes,
                                    ctypes.byref(h)))
    return Mesh(h, (len(hx), len(hy), len(hz)), p, lam)


# ---- MLP ------------------------------------------------------------------
def mlp_nparams(nout):
    return lib().pmg_mlp_nparams(nout)


def mlp_forward(params, x, y, cache, batch, nout, stream=None):
    _check(lib().pmg_mlp_forward(_ptr(params), _ptr(x), _ptr(y), _ptr(cache), batch, nout,
                                 _stream(stream)))


def mlp_loss(y, t, mask, dy, loss, batch, nout, stream=None):
    _check(lib().pmg_mlp_loss(_ptr(y), _ptr(t), _ptr(mask), _ptr(dy), _ptr(loss), batch, nout,
                              _stream(stream)))


def mlp_backward(params, x, cache, dy, grad, batch, nout, stream=None):
    _check(lib().pmg_mlp_backward(_ptr(params), _ptr(x), _ptr(cache), _ptr(dy), _ptr(grad), batch,
                                  nout, _stream(stream)))


def mlp_backward_noalloc(params, x, cache, dy, grad, batch, nout, stream=None):
    _check(lib().pmg_mlp_backward_noalloc(_ptr(params), _ptr(x), _ptr(cache), _ptr(dy), _ptr(grad),
                                          batch, nout, _stream(stream)))


def mlp_adam(params, grad, m, v, n, lr, beta1, beta2, eps, t, stream=None):
    _check(lib().pmg_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), n, lr, beta1, beta2,
                              eps, t, _stream(stream)))
