"""Python front end of libpfrac: mesh handles, device states and the staggered step.

Argument marshalling only: every step of the method runs in the HIP kernels
of libpfrac.  PyTorch provides device memory and the HIP stream.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

NODE_FIELDS = ("ux", "uy", "vx", "vy", "ax", "ay", "d")


def _stream(stream: torch.cuda.Stream | None = None) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def torch_dtype(code: str) -> torch.dtype:
    return {"f64": torch.float64, "f32": torch.float32}[code]


class Mesh:
    """A pf_mesh_t handle over one or more instances.

    ``meshes`` are objects with ``xy`` (N,2) float64, ``tri`` (Ne,3) int and
    ``fixed`` (N,2) uint8 arrays (for example workloads.Problem).
    """

    def __init__(self, meshes, dtype: str = "f64", tile_nodes: int = 0, device: str = "cuda",
                 explicit_block: int = 0, explicit_chunks: int = 0, damage_chunks: int = 0):
        if dtype not in ("f32", "f64"):
            raise ValueError(dtype)
        self.dtype_code = dtype
        self.dtype = torch_dtype(dtype)
        self.device = torch.device(device)
        # as requested (0: default)
        self.tile_nodes, self.explicit_block, self.explicit_chunks = int(tile_nodes), int(explicit_block), \
            int(explicit_chunks)
        n = len(meshes)
        keep = []
        descs = (L.MeshDesc * n)()
        for k, pr in enumerate(meshes):
            xy = np.ascontiguousarray(pr.xy, dtype=np.float64)
            tri = np.ascontiguousarray(pr.tri, dtype=np.int32)
            fx = None if getattr(pr, "fixed", None) is None else np.ascontiguousarray(pr.fixed, dtype=np.uint8)
            keep += [xy, tri, fx]
            descs[k] = L.MeshDesc(len(xy), len(tri), xy.ctypes.data, tri.ctypes.data,
                                  None if fx is None else fx.ctypes.data)
        h = C.c_void_p()
        opts = L.TileOpts(int(tile_nodes), int(explicit_block), int(explicit_chunks), int(damage_chunks))
        L.call("pf_mesh_create", descs, n, L.PF_F64 if dtype == "f64" else L.PF_F32, C.byref(opts),
               _stream(), C.byref(h))
        self.handle = h
        tot = L.Totals()
        L.call("pf_mesh_totals", h, C.byref(tot))
        self.totals = tot
        self.damage_chunks = int(tot.damage_chunks)   # as chosen by the library
        self.n_instances, self.n_nodes, self.n_elems = tot.n_instances, tot.n_nodes, tot.n_elems
        self.info = []
        for k in range(n):
            inf = L.InstanceInfo()
            L.call("pf_mesh_instance", h, k, C.byref(inf))
            self.info.append(inf)
        self.node_perm = np.empty(self.n_nodes, dtype=np.int32)
        L.call("pf_mesh_node_perm", h, self.node_perm.ctypes.data)
        self.elem_perm = np.empty(self.n_elems, dtype=np.int32)
        L.call("pf_mesh_elem_perm", h, self.elem_perm.ctypes.data)
        # internal position of every user node / element, per instance
        self.node_pos, self.elem_pos = [], []
        for inf in self.info:
            o, m = inf.node_offset, inf.n_nodes
            pos = np.empty(m, dtype=np.int64)
            pos[self.node_perm[o:o + m]] = np.arange(o, o + m)
            self.node_pos.append(pos)
            o, m = inf.elem_offset, inf.n_elems
            pos = np.empty(m, dtype=np.int64)
            pos[self.elem_perm[o:o + m]] = np.arange(o, o + m)
            self.elem_pos.append(pos)
        # toughness field Gc_e = Gc phi_e held by the handle (pf_set_gc_field)
        self.gc_scale: torch.Tensor | None = None
        self.gc_grad: torch.Tensor | None = None
        self.gc_version = 0

    def set_gc_field(self, scale: torch.Tensor | None, grad: torch.Tensor | None = None) -> None:
        """phi_e in internal element order (mesh dtype, device) or None for a uniform Gc;
        grad: float64 device tensor [n_elems] that pf_step_backward accumulates dL/dGc_e into."""
        same = scale is not None and scale is self.gc_scale   # re-registering the held field
        if scale is not None and not same:
            scale = scale.to(device=self.device, dtype=self.dtype).clone().contiguous()
            if scale.shape != (self.n_elems,):
                raise ValueError(f"toughness field must have {self.n_elems} values")
        if grad is not None and (grad.dtype != torch.float64 or grad.shape != (self.n_elems,)
                                 or grad.device.type != self.device.type or not grad.is_contiguous()):
            raise ValueError("grad must be a contiguous float64 device tensor of n_elems values")
        L.call("pf_set_gc_field", self.handle, _ptr(scale), _ptr(grad), _stream())
        if not same and (scale is not None or self.gc_scale is not None):
            self.gc_version += 1
        self.gc_scale, self.gc_grad = scale, grad

    def close(self) -> None:
        if getattr(self, "handle", None) is not None and self.handle.value:
            L.lib().pf_mesh_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- layout helpers (user numbering <-> internal numbering) ---------------
    def nodes_to_internal(self, per_inst) -> np.ndarray:
        first = np.asarray(per_inst[0])
        out = np.zeros((self.n_nodes,) + first.shape[1:], dtype=np.float64)
        for k, a in enumerate(per_inst):
            out[self.node_pos[k]] = np.asarray(a)
        return out

    def nodes_from_internal(self, arr) -> list:
        a = arr.detach().cpu().numpy() if isinstance(arr, torch.Tensor) else np.asarray(arr)
        return [a[pos] for pos in self.node_pos]

    def elems_to_internal(self, per_inst) -> np.ndarray:
        first = np.asarray(per_inst[0])
        out = np.zeros((self.n_elems,) + first.shape[1:], dtype=np.float64)
        for k, a in enumerate(per_inst):
            out[self.elem_pos[k]] = np.asarray(a)
        return out

    def elems_from_internal(self, arr) -> list:
        a = arr.detach().cpu().numpy() if isinstance(arr, torch.Tensor) else np.asarray(arr)
        return [a[pos] for pos in self.elem_pos]


class State:
    """Device state: node fields (7, N) = u_x u_y v_x v_y a_x a_y d, H (Ne) and the
    time t of every instance (float64; the explicit step advances it)."""

    def __init__(self, mesh: Mesh, nodes: torch.Tensor | None = None, H: torch.Tensor | None = None,
                 t: torch.Tensor | None = None):
        self.mesh = mesh
        self.nodes = nodes if nodes is not None else torch.zeros((7, mesh.n_nodes), dtype=mesh.dtype,
                                                                   device=mesh.device)
        self.H = H if H is not None else torch.zeros(mesh.n_elems, dtype=mesh.dtype, device=mesh.device)
        self.t = t if t is not None else torch.zeros(mesh.n_instances, dtype=torch.float64, device=mesh.device)

    def ptrs(self) -> L.StatePtrs:
        return L.StatePtrs(*[self.nodes[i].data_ptr() for i in range(7)], self.H.data_ptr(), self.t.data_ptr())

    def clone(self) -> "State":
        return State(self.mesh, self.nodes.clone(), self.H.clone(), self.t.clone())

    def copy_(self, other: "State") -> "State":
        self.nodes.copy_(other.nodes)
        self.H.copy_(other.H)
        self.t.copy_(other.t)
        return self

    def zero_(self) -> "State":
        self.nodes.zero_()
        self.H.zero_()
        self.t.zero_()
        return self

    @property
    def d(self) -> torch.Tensor:
        return self.nodes[6]

    def to_user(self) -> list[dict]:
        """Per instance: dict of numpy arrays u, v, a (N,2), d (N,), H (Ne,) in the caller's numbering."""
        nodes = self.mesh.nodes_from_internal(self.nodes.double().T)
        H = self.mesh.elems_from_internal(self.H.double())
        out = []
        for k in range(self.mesh.n_instances):
            nd = nodes[k]
            out.append({"u": nd[:, 0:2], "v": nd[:, 2:4], "a": nd[:, 4:6], "d": nd[:, 6], "H": H[k]})
        return out

    @staticmethod
    def from_user(mesh: Mesh, per_inst: list[dict]) -> "State":
        cols = [np.concatenate([np.asarray(s["u"]), np.asarray(s["v"]), np.asarray(s["a"]),
                                np.asarray(s["d"])[:, None]], 1) for s in per_inst]
        nodes = torch.tensor(mesh.nodes_to_internal(cols).T.copy(), dtype=mesh.dtype, device=mesh.device)
        H = torch.tensor(mesh.elems_to_internal([np.asarray(s["H"]) for s in per_inst]), dtype=mesh.dtype,
                         device=mesh.device)
        return State(mesh, nodes.contiguous(), H)


def params_of(problem, Gc: float | None = None) -> L.Params:
    return L.Params(problem.E, problem.nu, problem.rho, problem.Gc if Gc is None else Gc, problem.l0, problem.eta,
                    problem.gamma_star, int(problem.model), L.SPLITS[problem.split], L.PLANES[problem.plane],
                    L.BOUNDS[getattr(problem, "bounds", "projected")])


@dataclass
class CgConfig:
    tol: float = 1e-12
    max_iter: int = 2000
    check_every: int = 8
    start: int = 1          # damage solve: 1 = extrapolate from the two previous damage fields
    monotone: int = 0       # damage solve: 1 = monotone projected CG from the start
    rounds: int = 0         # check_every = 0: CG rounds to enqueue (0 = max_iter)
    resume: int = 0         # damage solve: 1 = continue the handle's previous solve
    precond: int = 0        # 0: Jacobi; 2-4: Chebyshev-Jacobi polynomial of that degree

    def opts(self) -> L.CgOpts:
        return L.CgOpts(self.tol, self.max_iter, self.check_every, self.start, self.monotone, self.rounds,
                        self.resume, self.precond)


def default_tol(dtype: str) -> float:
    return 1e-12 if dtype == "f64" else 1e-6


class Loading:
    """Ramped boundary loads of a Simulator (Sec. 3 loading protocols), held by the library.

    traction: per instance an (N, 2) nodal force reached at full load (or
    None); the explicit step ending at t_{n+1} applies S(t_{n+1}) F, with S
    the smooth ramp of time t_traction.  t_velocity > 0 ramps the prescribed
    velocities (the problems' v0 on their fixed DOFs) linearly up to v0 over
    t_velocity, evaluated at each step's midpoint.  This class only converts
    the arrays to the library's node order and registers them
    (pf_set_loading); the ramps are evaluated in the explicit-step kernel from
    the state time.
    """

    def __init__(self, sim: "Simulator", traction=None, t_traction: float = 0.0, t_velocity: float = 0.0):
        mesh = sim.mesh
        self.t_traction = float(t_traction)
        self.t_velocity = float(t_velocity)
        F = v0 = None
        if traction is not None:
            per = traction if isinstance(traction, (list, tuple)) else [traction]
            F = torch.tensor(mesh.nodes_to_internal([np.asarray(f, dtype=np.float64) for f in per]).T.copy(),
                             dtype=mesh.dtype, device=mesh.device)                   # (2, N)
        if self.t_velocity > 0.0:
            v0 = torch.tensor(mesh.nodes_to_internal([np.asarray(p.v0, dtype=np.float64)
                                                      for p in sim.problems]).T.copy(),
                              dtype=mesh.dtype, device=mesh.device)
        n = mesh.n_instances
        tf = (C.c_double * n)(*([self.t_traction] * n))
        tv = (C.c_double * n)(*([self.t_velocity] * n))
        L.call("pf_set_loading", mesh.handle, _ptr(F), _ptr(v0), tf, tv, _stream())


class Simulator:
    """Staggered explicit phase-field simulation of one or more instances on one GPU."""

    def __init__(self, problems, dtype: str | None = None, tile_nodes: int | str = 0, cg: CgConfig | None = None,
                 dt: list[float] | None = None, mesh: Mesh | None = None, cg_adj: CgConfig | None = None,
                 n_sub: int = 1, allow_beyond_limit: bool = False):
        if not isinstance(problems, (list, tuple)):
            problems = [problems]
        self.problems = list(problems)
        self.dtype_code = dtype or self.problems[0].dtype
        explicit_block = explicit_chunks = 0
        if mesh is None and tile_nodes == "auto":
            from .tune import tune_tiles
            rep = tune_tiles(self.problems, self.dtype_code)
            tile_nodes, explicit_block, explicit_chunks = rep["best"], rep["explicit_block"], rep["explicit_chunks"]
        self.mesh = mesh or Mesh(self.problems, self.dtype_code, tile_nodes, explicit_block=explicit_block,
                                 explicit_chunks=explicit_chunks)
        n = len(self.problems)
        self.params = (L.Params * n)(*[params_of(p) for p in self.problems])
        self.dt = (C.c_double * n)()
        if dt is None:
            cfl = self.problems[0].cfl
            if any(p.cfl != cfl for p in self.problems):
                raise ValueError("all instances of a simulator share one CFL factor")
            L.call("pf_cfl_dt", self.mesh.handle, self.params, cfl, self.dt)
        else:
            for k, v in enumerate(dt):
                self.dt[k] = float(v)
        # damage subcycling (Sec. 2.3): the damage sub-problem is solved on
        # every n_sub-th step; the pre-simulation check computes N_max
        nmax = (C.c_int32 * n)()
        ratio = (C.c_double * n)()
        L.call("pf_subcycle_limit", self.mesh.handle, self.params, nmax, ratio)
        self.n_max = [int(v) for v in nmax]
        self.subcycle_ratio = [float(v) for v in ratio]
        if int(n_sub) < 1:
            raise ValueError("n_sub must be >= 1")
        if int(n_sub) > min(self.n_max) and not allow_beyond_limit:
            raise ValueError(f"n_sub = {n_sub} exceeds N_max = {min(self.n_max)} "
                             f"(c_p / (0.6 c_R) = {min(self.subcycle_ratio):.3f})")
        self.n_sub = int(n_sub)
        self.cg = cg or CgConfig(tol=default_tol(self.dtype_code))
        # adjoint solves stop relative to their right-hand side
        self.cg_adj = cg_adj or CgConfig(tol=default_tol(self.dtype_code))
        self.window_redos = 0   # windows of run() re-run with polling (a solve outran its budget)
        self.stats = torch.zeros(n * 6, dtype=torch.int32, device=self.mesh.device)   # pf_cg_stats_t[n]
        self.active = self.initial_active()
        self._active_next = torch.zeros_like(self.active)
        self.state = self.initial_state()
        self._next = State(self.mesh)
        self.steps_done = 0
        self.loading: Loading | None = None

    def set_loading(self, traction=None, t_traction: float = 0.0, t_velocity: float = 0.0) -> None:
        """Ramped loads for the following steps (see Loading); no arguments clears them."""
        if traction is None and t_velocity <= 0.0:
            L.call("pf_set_loading", self.mesh.handle, None, None, None, None, _stream())
            self.loading = None
        else:
            self.loading = Loading(self, traction, t_traction, t_velocity)

    def set_Gc(self, values) -> None:
        for k, v in enumerate(np.atleast_1d(values)):
            self.params[k].Gc = float(v)

    def set_gc_field(self, fields=None) -> None:
        """Spatially varying toughness Gc_e = Gc phi_e: one array of phi_e per
        instance in the user's element order (None: uniform Gc)."""
        if fields is None:
            self.mesh.set_gc_field(None, self.mesh.gc_grad)
            return
        if len(fields) != self.mesh.n_instances:
            raise ValueError("one toughness field per instance")
        phi = torch.tensor(self.mesh.elems_to_internal([np.asarray(f, dtype=np.float64) for f in fields]),
                           dtype=self.mesh.dtype, device=self.mesh.device)
        self.mesh.set_gc_field(phi, self.mesh.gc_grad)

    def initial_state(self) -> State:
        return State.from_user(self.mesh, [{"u": p.u0, "v": p.v0, "a": p.a0, "d": p.d0, "H": p.H0}
                                           for p in self.problems])

    def initial_active(self) -> torch.Tensor:
        """Held-set seed for the first solve: nodes whose initial damage is already 1 (the notch)."""
        d0 = self.mesh.nodes_to_internal([p.d0 for p in self.problems])
        return torch.tensor((d0 >= 1.0).astype(np.uint8), device=self.mesh.device)

    def reset(self) -> None:
        self.state = self.initial_state()
        self.active = self.initial_active()
        self._next.zero_()
        self.steps_done = 0

    # --- the two halves of the staggered step --------------------------------
    def explicit(self, s_in: State, s_out: State, f_ext: torch.Tensor | None = None) -> None:
        a, b = s_in.ptrs(), s_out.ptrs()
        L.call("pf_explicit_step", self.mesh.handle, self.params, self.dt, C.byref(a), C.byref(b),
               _ptr(f_ext), _stream())

    def damage(self, H: torch.Tensor, d_prev: torch.Tensor, d_out: torch.Tensor,
               active: torch.Tensor | None = None, guess: torch.Tensor | None = None,
               cg: CgConfig | None = None, stats: torch.Tensor | None = None) -> None:
        """Damage update; `guess` seeds the held set (normally the previous step's flags)."""
        o = (cg or self.cg).opts()
        L.call("pf_damage_solve", self.mesh.handle, self.params, H.data_ptr(), d_prev.data_ptr(), d_out.data_ptr(),
               _ptr(guess), _ptr(active), C.byref(o), (stats if stats is not None else self.stats).data_ptr(),
               _stream())

    def step_into(self, s_in: State, s_out: State, active_out: torch.Tensor, active_in: torch.Tensor | None,
                  f_ext: torch.Tensor | None = None) -> None:
        """One staggered step s_in -> s_out; active_in are the flags of the solve that produced s_in.d.

        With the extrapolated start (cg.start = 1), s_out.d must hold the damage
        of the step before s_in on entry; the explicit step leaves it untouched.
        """
        self.explicit(s_in, s_out, f_ext)
        self.damage(s_out.H, s_in.d, s_out.d, active_out, active_in)

    def solves_at(self, step_index: int) -> bool:
        """Whether step number step_index (0-based) solves the damage sub-problem."""
        return (step_index + 1) % self.n_sub == 0

    def skip_into(self, s_in: State, s_out: State, f_ext: torch.Tensor | None = None) -> None:
        """A step without the damage solve (subcycling): explicit step, then d_{n+1} = d_n."""
        self.explicit(s_in, s_out, f_ext)
        s_out.d.copy_(s_in.d)

    def step(self, n: int = 1, rounds_out: list | None = None) -> State:
        """n staggered steps, each damage solve polled for convergence; rounds_out, if given,
        receives each solve's CG round count (the largest over the instances)."""
        for _ in range(n):
            if self.solves_at(self.steps_done):
                self.step_into(self.state, self._next, self._active_next, self.active)
                self.active, self._active_next = self._active_next, self.active
                if rounds_out is not None:
                    rounds_out.append(max(s["iters"] for s in self.cg_stats()))
            else:
                self.skip_into(self.state, self._next)
            self.state, self._next = self._next, self.state
            self.steps_done += 1
        return self.state

    def run(self, n: int, window: int = 16, margin: int = 2, rounds_out: list | None = None) -> State:
        """n staggered steps with the solver's convergence read once per window of steps.

        Each step enqueues the explicit step and a fixed budget of CG rounds
        (check_every = 0, so the host never waits inside a step); the budget
        is the largest round count of the previous window's last eight solves
        plus `margin` (the first steps of a simulator run polled, to learn
        it).  After a window the per-step statistics are read once: if a
        solve did not finish within its budget, the window is rolled back to
        its first state and re-run with step(), which polls.  Rounds after a
        solve has finished do nothing, so the states equal those of step(n)
        bit for bit.  rounds_out, if given, receives each solve's CG round count
        (the largest over the instances), in step order.
        """
        ni = self.mesh.n_instances
        if getattr(self, "_win_stats", None) is None or self._win_stats.shape[0] < window:
            self._win_stats = torch.zeros((window, ni * 6), dtype=torch.int32, device=self.mesh.device)
        budget = getattr(self, "_budget", 0)
        done = 0
        if not budget:
            # no round counts seen yet: the first steps poll
            k = min(4, n)
            its = []
            for _ in range(k):
                self.step()
                if self.solves_at(self.steps_done - 1):
                    its.append(max(s["iters"] for s in self.cg_stats()))
                    if rounds_out is not None:
                        rounds_out.append(its[-1])
            budget = (max(its) + margin) if its else 0
            done = k
        while done < n:
            w = min(window, n - done)
            if not budget:
                self.step(w, rounds_out)
                its = [s["iters"] for s in self.cg_stats()]
                budget = max(its) + margin if any(self.solves_at(self.steps_done - 1 - j) for j in range(w)) else 0
                done += w
                continue
            refs = (self.state, self._next, self.active, self._active_next)
            snap = (self.state.clone(), self._next.d.clone(), self.active.clone())
            o = C.byref(CgConfig(self.cg.tol, self.cg.max_iter, 0, self.cg.start, self.cg.monotone,
                                 min(budget, self.cg.max_iter), 0, self.cg.precond).opts())
            solved = []
            for k in range(w):
                if not self.solves_at(self.steps_done + k):
                    self.skip_into(self.state, self._next)
                    self.state, self._next = self._next, self.state
                    continue
                self.explicit(self.state, self._next)
                L.call("pf_damage_solve", self.mesh.handle, self.params, self._next.H.data_ptr(),
                       self.state.d.data_ptr(), self._next.d.data_ptr(), self.active.data_ptr(),
                       self._active_next.data_ptr(), o, self._win_stats[k].data_ptr(), _stream())
                self.state, self._next = self._next, self.state
                self.active, self._active_next = self._active_next, self.active
                solved.append(k)
            st = self._win_stats[:w].cpu().numpy().reshape(w, ni, 6)[solved]
            if len(solved) == 0:
                self.steps_done += w
            elif np.any(st[:, :, 3] != 0):
                # a solve did not finish within the budget: redo the window, polling
                self.window_redos += 1
                self.state, self._next, self.active, self._active_next = refs
                self.state.copy_(snap[0])
                self._next.d.copy_(snap[1])
                self.active.copy_(snap[2])
                self.step(w, rounds_out)
                budget = max(s["iters"] for s in self.cg_stats()) + 2 * margin
            else:
                self.stats.copy_(self._win_stats[solved[-1]])
                self.steps_done += w
                budget = int(st[-8:, :, 0].max()) + margin
                if rounds_out is not None:
                    rounds_out.extend(int(r) for r in st[:, :, 0].max(axis=1))
            done += w
        self._budget = budget
        return self.state

    def energies(self, state: State | None = None, out: torch.Tensor | None = None,
                 static_scratch: bool = False) -> list[tuple[float, float, float]]:
        """(E_kin, E_el, E_frac) of every instance, per unit thickness (pf_energies, or with
        static_scratch pf_energies_static, whose partial sums live in the library's fixed
        device array; `out`, a device double tensor of 3 n_instances entries, receives them)."""
        st = state or self.state
        if out is None:
            out = torch.empty(self.mesh.n_instances * 3, dtype=torch.float64, device=self.mesh.device)
        ptrs = st.ptrs()
        L.call("pf_energies_static" if static_scratch else "pf_energies", self.mesh.handle, self.params,
               C.byref(ptrs), out.data_ptr(), _stream())
        e = out.cpu().numpy().reshape(-1, 3)
        return [tuple(float(x) for x in r) for r in e]

    def cg_stats(self) -> list[dict]:
        raw = self.stats.cpu().numpy().view(np.int32).reshape(-1, 6)
        out = []
        for r in raw:
            resid = np.frombuffer(r[4:6].tobytes(), dtype=np.float64)[0]
            out.append({"iters": int(r[0]), "restarts": int(r[1]), "n_active": int(r[2]), "flags": int(r[3]),
                        "resid": float(resid)})
        return out

    def repeat_damage_pass(self, n: int, H: torch.Tensor, d_prev: torch.Tensor, d: torch.Tensor) -> None:
        """n back-to-back launches of the damage pass the last solve stopped at (pf_damage_pass_repeat);
        H, d_prev and d are the arrays that solve was given."""
        L.call("pf_damage_pass_repeat", self.mesh.handle, H.data_ptr(), d_prev.data_ptr(), d.data_ptr(), int(n),
               _stream())

    def timer(self, on: bool) -> None:
        L.call("pf_timer_enable", self.mesh.handle, 1 if on else 0)

    def timer_read(self, family: int) -> tuple[float, int]:
        ms = C.c_double()
        n = C.c_int64()
        L.call("pf_timer_read", self.mesh.handle, family, C.byref(ms), C.byref(n))
        return ms.value, n.value


class GraphStepper:
    """Staggered steps of a Simulator replayed from HIP graphs.

    For each direction of the simulator's ping-pong state pair, one graph holds
    the explicit step and the first `rounds` rounds of the damage solve, and a
    second graph `more` further rounds (resume).  A step replays the first
    graph, reads the per-instance CG statistics once, and replays the second
    until every instance has finished, so results equal Simulator.step bit for
    bit.  The material parameters, toughness field and time steps are those
    of the capture; build a new stepper after changing them.
    """

    def __init__(self, sim: Simulator, rounds: int | None = None, more: int = 4):
        if sim.n_sub != 1:
            raise NotImplementedError("graph replay covers the step with a damage solve (n_sub = 1)")
        self.sim = sim
        base = sim.cg
        self.max_iter = base.max_iter
        # one eager step so the device holds this simulator's parameters (a
        # captured call must not upload anything); by default the first graph
        # holds four rounds more than that step's solve needed
        sim.step()
        torch.cuda.synchronize()
        if rounds is None:
            rounds = max(s["iters"] for s in sim.cg_stats()) + 4
        self.rounds, self.more = rounds, more
        first = CgConfig(base.tol, base.max_iter, 0, base.start, base.monotone, rounds, 0, base.precond)
        cont = CgConfig(base.tol, base.max_iter, 0, base.start, base.monotone, more, 1, base.precond)
        self._params = bytes(sim.params)
        self._dt = list(sim.dt)
        self._gc_version = sim.mesh.gc_version
        self.states = (sim.state, sim._next)
        self.actives = (sim.active, sim._active_next)
        self.graphs = []
        for k in (0, 1):
            s_in, s_out = self.states[k], self.states[1 - k]
            a_in, a_out = self.actives[k], self.actives[1 - k]
            g1, g2 = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
            with torch.cuda.graph(g1):
                sim.explicit(s_in, s_out)
                sim.damage(s_out.H, s_in.d, s_out.d, a_out, a_in, cg=first)
            with torch.cuda.graph(g2):
                sim.damage(s_out.H, s_in.d, s_out.d, a_out, a_in, cg=cont)
            self.graphs.append((g1, g2))
        self.parity = 0
        self.continuations = 0

    def step(self, n: int = 1) -> State:
        sim = self.sim
        if bytes(sim.params) != self._params or list(sim.dt) != self._dt \
                or sim.mesh.gc_version != self._gc_version:
            raise RuntimeError("parameters changed since the graphs were captured")
        for _ in range(n):
            g1, g2 = self.graphs[self.parity]
            g1.replay()
            while True:
                st = sim.stats.cpu().numpy().view(np.int32).reshape(-1, 6)
                if not np.any(st[:, 3] & L.PF_FLAG_NONFINITE) and not np.any(st[:, 3] & L.PF_FLAG_NOT_CONVERGED):
                    break
                if np.any(st[:, 3] & L.PF_FLAG_NONFINITE):
                    raise L.PfError(L.PF_ERR_NONFINITE, "GraphStepper.step", "non-finite value in the damage CG")
                if np.any(st[:, 0] >= self.max_iter):
                    raise L.PfError(L.PF_ERR_NOT_CONVERGED, "GraphStepper.step", "damage CG reached max_iter")
                g2.replay()
                self.continuations += 1
            self.parity ^= 1
            sim.state, sim._next = self.states[self.parity], self.states[1 - self.parity]
            sim.active, sim._active_next = self.actives[self.parity], self.actives[1 - self.parity]
            sim.steps_done += 1
        return sim.state
