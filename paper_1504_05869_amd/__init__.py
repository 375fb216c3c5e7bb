"""lkp: higher-order lattice-kinetic Poisson solver for AMD MI355X (gfx950).

Thin binding over the C ABI of ``include/lkp.h`` (``liblkp.so``, built in-tree
with hipcc).  Every step of the solver runs in the library's HIP kernels; this
module only marshals arguments.  PyTorch provides device memory and streams.

    import paper_1504_05869_amd as lkp
    p = lkp.Problem(source, lattice="D2Q81", order=5, knudsen=0.1)
    rep = p.solve(tol_rel_l2=1e-10)
    phi = p.phi()            # torch tensor on the GPU, FP64
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import LATTICES, PRECISIONS, LkpError, check

__all__ = ["Problem", "Group", "lattice_info", "footprint_bytes", "contraction_bound", "LkpError",
           "LATTICES", "PRECISIONS", "library_path", "solve_opts"]


def library_path() -> str:
    return _lib.LIB_PATH


def _stream_handle(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _desc(shape, lattice, order, tau_lb, knudsen, precision, subtract_mean, allow_unstable):
    if lattice not in LATTICES:
        raise ValueError(f"unknown lattice {lattice!r}")
    if precision not in PRECISIONS:
        raise ValueError(f"unknown precision {precision!r}")
    if (tau_lb is None) == (knudsen is None):
        raise ValueError("give exactly one of tau_lb and knudsen")
    d = _lib.ProblemDesc()
    d.dim = len(shape)
    n = list(shape)[::-1] + [1] * (3 - len(shape))   # (nz, ny, nx) -> nx, ny, nz
    for a in range(3):
        d.n[a] = int(n[a])
    d.lattice = LATTICES[lattice]
    d.order = int(order)
    d.precision = PRECISIONS[precision]
    d.tau_lb = float(tau_lb) if tau_lb is not None else 0.0
    d.knudsen = float(knudsen) if knudsen is not None else 0.0
    d.subtract_mean = int(bool(subtract_mean))
    d.allow_unstable = int(bool(allow_unstable))
    return d


def footprint_bytes(shape, lattice, order, tau_lb=None, knudsen=None, precision="f64",
                    in_place=False, population_sweep=False) -> int:
    """Device bytes of the state of a problem of this description, which is
    also the smallest workspace it accepts (0 if invalid)."""
    d = _desc(shape, lattice, order, tau_lb, knudsen, precision, False, True)
    d.flags = ((_lib.FLAG_IN_PLACE if in_place else 0)
               | (_lib.FLAG_POPULATION_SWEEP if population_sweep else 0))
    return int(_lib.load().lkp_footprint_bytes(ctypes.byref(d)))


def contraction_bound(shape, lattice, order, tau_lb=None, knudsen=None, drift=None) -> float:
    """Slowest decay the sweep allows on this grid (lkp_contraction_bound)."""
    d = _desc(shape, lattice, order, tau_lb, knudsen, "f64", False, True)
    if drift is not None:
        for a, u in enumerate(drift):
            d.drift[a] = float(u)
    rho = ctypes.c_double()
    check(_lib.load().lkp_contraction_bound(ctypes.byref(d), ctypes.byref(rho)),
          "lkp_contraction_bound")
    return float(rho.value)


def lattice_info(lattice: str, order: int = 1) -> dict:
    """Velocities, weights, phi_i, chi_i and c_s^2 the library uses."""
    lib = _lib.load()
    q, dim = ctypes.c_int32(), ctypes.c_int32()
    v = np.zeros((169, 3), dtype=np.int32)
    w, ph, ch = (np.zeros(169) for _ in range(3))
    cs2 = ctypes.c_double()
    check(lib.lkp_lattice_info(LATTICES[lattice], int(order), ctypes.byref(q), ctypes.byref(dim),
                               v.ctypes.data, w.ctypes.data, ph.ctypes.data, ch.ctypes.data,
                               ctypes.byref(cs2)), "lkp_lattice_info")
    Q = q.value
    return {"Q": Q, "dim": dim.value, "v": v[:Q].copy(), "w": w[:Q].copy(),
            "phi": ph[:Q].copy(), "chi": ch[:Q].copy(), "cs2": cs2.value}


def solve_opts(tol_rel_l2=0.0, tol_maxchange=0.0, max_sweeps=10_000_000, check_every=100,
               use_graph=True, max_outer=0, ir_inner_tol=0.0) -> _lib.SolveOpts:
    o = _lib.SolveOpts()
    o.tol_rel_l2 = float(tol_rel_l2)
    o.tol_maxchange = float(tol_maxchange)
    o.max_sweeps = int(max_sweeps)
    o.check_every = int(check_every)
    o.use_graph = int(bool(use_graph))
    o.max_outer = int(max_outer)
    o.ir_inner_tol = float(ir_inner_tol)
    return o


class Problem:
    """One resident periodic Poisson problem lap(Phi) = -s on the GPU."""

    def __init__(self, source, lattice: str, order: int, tau_lb=None, knudsen=None,
                 precision: str = "f64", subtract_mean: bool = False,
                 allow_unstable: bool = False, stream=None, population_sweep: bool = False,
                 in_place: bool = False, drift=None, workspace=None):
        """drift: uniform drift (ux, uy, uz) in velocity-component order (x is the
        last array axis) for the advection-diffusion variant; None = diffusion.

        workspace: None, the library allocates the device state; True, the
        state is placed in a byte tensor taken from torch's caching allocator
        (freed back to torch when the problem closes); or a contiguous CUDA
        tensor of at least ``footprint_bytes`` bytes, 256-byte aligned, that the
        caller keeps and does not touch while the problem is open."""
        self._lib = _lib.load()
        self._h = ctypes.c_void_p()
        if isinstance(source, torch.Tensor):
            src = source.detach().to(torch.float64).contiguous()
            shape = tuple(src.shape)
            on_dev = src.is_cuda
            ptr = src.data_ptr()
        else:
            src = np.ascontiguousarray(source, dtype=np.float64)
            shape = src.shape
            on_dev = False
            ptr = src.ctypes.data
        self.shape = tuple(int(s) for s in shape)
        d = _desc(self.shape, lattice, order, tau_lb, knudsen, precision, subtract_mean,
                  allow_unstable)
        d.source = ptr
        d.source_on_device = int(on_dev)
        d.flags = ((_lib.FLAG_POPULATION_SWEEP if population_sweep else 0)
                   | (_lib.FLAG_IN_PLACE if in_place else 0))
        self._stream = _stream_handle(stream)
        d.stream = self._stream
        if drift is not None:
            u = [float(x) for x in drift]
            if len(u) > 3:
                raise ValueError("drift has at most 3 components")
            for a, x in enumerate(u):
                d.drift[a] = x
        self.lattice, self.order, self.precision = lattice, int(order), precision
        self._ws = None
        if workspace is not None and workspace is not False:
            need = int(self._lib.lkp_footprint_bytes(ctypes.byref(d)))
            if need <= 0:
                check(self._lib.lkp_create(ctypes.byref(d), ctypes.byref(self._h)), "lkp_create")
            if workspace is True:
                ws = torch.empty(need, dtype=torch.uint8, device="cuda")
            else:
                ws = workspace
                if not (isinstance(ws, torch.Tensor) and ws.is_cuda and ws.is_contiguous()):
                    raise ValueError("workspace must be a contiguous CUDA tensor")
            d.workspace = ws.data_ptr()
            d.workspace_bytes = ws.numel() * ws.element_size()
            self._ws = ws
        check(self._lib.lkp_create(ctypes.byref(d), ctypes.byref(self._h)), "lkp_create")
        del src

    # ------------------------------------------------------------ lifecycle
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.lkp_destroy(self._h)
            self._h = ctypes.c_void_p()
        self._ws = None   # the workspace outlives the handle

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------- compute
    def step(self, sweeps: int):
        check(self._lib.lkp_step(self._h, int(sweeps)), "lkp_step")

    def solve(self, tol_rel_l2: float = 0.0, tol_maxchange: float = 0.0,
              max_sweeps: int = 10_000_000, check_every: int = 100, use_graph: bool = True,
              max_outer: int = 0, ir_inner_tol: float = 0.0, raise_on_error: bool = True) -> dict:
        o = solve_opts(tol_rel_l2, tol_maxchange, max_sweeps, check_every, use_graph, max_outer,
                       ir_inner_tol)
        r = _lib.SolveReport()
        st = self._lib.lkp_solve(self._h, ctypes.byref(o), ctypes.byref(r))
        rep = {f: getattr(r, f) for f, _ in _lib.SolveReport._fields_}
        if st != 0 and raise_on_error:
            raise LkpError(st, "lkp_solve")
        return rep

    def residual(self) -> dict:
        r = _lib.ResidualReport()
        check(self._lib.lkp_residual(self._h, ctypes.byref(r)), "lkp_residual")
        return {f: getattr(r, f) for f, _ in _lib.ResidualReport._fields_}

    def sync(self):
        check(self._lib.lkp_sync(self._h), "lkp_sync")

    # ---------------------------------------------------------- read-back
    def phi(self, out: torch.Tensor | None = None) -> torch.Tensor:
        """Phi of the last sweep as an FP64 tensor on the GPU (shape of the source)."""
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device="cuda")
        assert out.is_cuda and out.dtype == torch.float64 and out.is_contiguous()
        assert out.numel() == int(np.prod(self.shape))
        check(self._lib.lkp_get_phi(self._h, out.data_ptr(), 1), "lkp_get_phi")
        return out

    def phi_host(self) -> np.ndarray:
        out = np.empty(self.shape, dtype=np.float64)
        check(self._lib.lkp_get_phi(self._h, out.ctypes.data, 0), "lkp_get_phi")
        return out

    def populations(self) -> np.ndarray:
        info = self.info()
        out = np.empty((info["Q"],) + self.shape, dtype=np.float64)
        check(self._lib.lkp_get_populations(self._h, out.ctypes.data, 0), "lkp_get_populations")
        return out

    def set_populations(self, f) -> None:
        f = np.ascontiguousarray(f, dtype=np.float64)
        check(self._lib.lkp_set_populations(self._h, f.ctypes.data, 0), "lkp_set_populations")

    def coefficients(self):
        """(phi_i, chi_i) of this handle, in lattice_info's velocity order."""
        q = self.info()["Q"]
        phi, chi = np.empty(q), np.empty(q)
        check(self._lib.lkp_get_coefficients(self._h, phi.ctypes.data, chi.ctypes.data),
              "lkp_get_coefficients")
        return phi, chi

    def set_equilibrium(self, phi0) -> None:
        """Start a time-dependent run from the equilibrium f*_i = phi_i Phi_0
        (formed on the device by the library)."""
        if isinstance(phi0, torch.Tensor) and phi0.is_cuda:
            t = phi0.detach().to(torch.float64).contiguous()
            if tuple(t.shape) != self.shape:
                raise ValueError("Phi_0 must have the problem's shape")
            check(self._lib.lkp_set_equilibrium(self._h, t.data_ptr(), 1), "lkp_set_equilibrium")
            return
        a = np.ascontiguousarray(phi0, dtype=np.float64)
        if a.shape != self.shape:
            raise ValueError("Phi_0 must have the problem's shape")
        check(self._lib.lkp_set_equilibrium(self._h, a.ctypes.data, 0), "lkp_set_equilibrium")

    def info(self) -> dict:
        i = _lib.HandleInfo()
        check(self._lib.lkp_get_info(self._h, ctypes.byref(i)), "lkp_get_info")
        d = {f: getattr(i, f) for f, _ in _lib.HandleInfo._fields_}
        d["n"] = tuple(i.n)
        return d


class Group:
    """Resident problems of one class advanced together in batched sweeps."""

    def __init__(self, lattice: str, order: int, precision: str = "f64", stream=None):
        self._lib = _lib.load()
        self._g = ctypes.c_void_p()
        self._stream = _stream_handle(stream)
        self.lattice, self.order, self.precision = lattice, int(order), precision
        check(self._lib.lkp_group_create(LATTICES[lattice], int(order), PRECISIONS[precision],
                                         self._stream, ctypes.byref(self._g)), "lkp_group_create")
        self._members = {}

    def add(self, problem: Problem, tol_rel_l2=0.0, tol_maxchange=0.0, max_sweeps=10_000_000):
        o = solve_opts(tol_rel_l2, tol_maxchange, max_sweeps)
        check(self._lib.lkp_group_add(self._g, problem._h, ctypes.byref(o)), "lkp_group_add")
        self._members[problem._h.value] = problem

    def remove(self, problem: Problem):
        check(self._lib.lkp_group_remove(self._g, problem._h), "lkp_group_remove")
        self._members.pop(problem._h.value, None)

    def __len__(self):
        return len(self._members)

    def step(self, sweeps: int) -> list:
        """Advance every running member; returns one report dict per member."""
        cap = max(1, len(self._members))
        arr = (_lib.MemberReport * cap)()
        n = ctypes.c_int32()
        check(self._lib.lkp_group_step(self._g, int(sweeps), arr, cap, ctypes.byref(n)),
              "lkp_group_step")
        out = []
        for k in range(min(n.value, cap)):
            r = arr[k]
            out.append({"problem": self._members.get(r.handle), "state": _lib.MEMBER_STATES[r.state],
                        "status": _lib.STATUS.get(r.status, r.status), "sweeps": r.sweeps,
                        "outer": r.outer, "est_rel_err": r.est_rel_err,
                        "max_change": r.max_change, "phi_l2": r.phi_l2})
        return out

    def split(self) -> int:
        """Velocity-group split of the group's batched sweeps (chosen at its
        first step with enough work)."""
        P = ctypes.c_int32()
        check(self._lib.lkp_group_split(self._g, ctypes.byref(P)), "lkp_group_split")
        return P.value

    def graph_stats(self) -> dict:
        """Graphs captured and steps replayed from a graph so far."""
        c, r = ctypes.c_int64(), ctypes.c_int64()
        check(self._lib.lkp_group_graph_stats(self._g, ctypes.byref(c), ctypes.byref(r)),
              "lkp_group_graph_stats")
        return {"captures": c.value, "replays": r.value}

    def close(self):
        if getattr(self, "_g", None) and self._g.value:
            self._lib.lkp_group_destroy(self._g)
            self._g = ctypes.c_void_p()
            self._members.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
