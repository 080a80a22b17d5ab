"""Python front end of one or many periodic LJ boxes on one GPU.

PyTorch provides device memory (the library's workspace and the caller's
arrays) and the stream (torch's current stream); every step of the method
runs in the HIP library through the C ABI in ``_abi``.
"""

from __future__ import annotations

from typing import Sequence

import torch

from . import _abi as abi
from . import tune_cache


def _stream() -> int:
    return int(torch.cuda.current_stream().cuda_stream)


def _require_cuda():
    if not torch.cuda.is_available():
        raise RuntimeError("paper_2009_07400_amd needs a ROCm GPU (torch.cuda.is_available() is False)")


def _soa(t, n: int, device) -> torch.Tensor:
    """[N,3] or [3,N] -> contiguous float64 [3,N] on the device."""
    t = torch.as_tensor(t, dtype=torch.float64, device=device)
    if t.shape == (n, 3):
        t = t.t()
    if t.shape != (3, n):
        raise ValueError(f"expected shape ({n}, 3) or (3, {n}), got {tuple(t.shape)}")
    return t.contiguous()


def _ptrs(t3: torch.Tensor):
    return [int(t3[k].data_ptr()) for k in range(3)]


_MODELS = {"lj": abi.TMD_MODEL_LJ, "spring_dashpot": abi.TMD_MODEL_SPRING_DASHPOT}


def make_params(epsilon=1.0, sigma=1.0, mass=1.0, cutoff=2.5, skin=0.3, dt=0.005, rebuild_every=20,
                max_neighbors=128, model="lj", stiffness=0.0, damping=0.0) -> abi.TmdParams:
    """model "lj" (Eq. 2) or "spring_dashpot" (Eq. 3: spheres of diameter
    sigma, spring constant stiffness, dissipation damping)."""
    if model not in _MODELS:
        raise ValueError(f"model must be one of {sorted(_MODELS)}")
    return abi.TmdParams(epsilon, sigma, mass, cutoff, skin, dt, rebuild_every, max_neighbors, stiffness, damping,
                         _MODELS[model], 0)


def compute_forces_static(pos, box_length: float, device="cuda", **params):
    """One-shot forces of one periodic box through tmd_compute_forces_static,
    whose intermediates live in the library's own device array (no
    workspace).  pos: [N, 3].  Returns (F [N, 3], [U, W], status [2] int32),
    all device tensors written on torch's current stream."""
    abi.load_library()
    _require_cuda()
    n = int(torch.as_tensor(pos).shape[0])
    p = _soa(pos, n, device)
    f = torch.empty(3, n, dtype=torch.float64, device=device)
    ev = torch.empty(2, dtype=torch.float64, device=device)
    st = torch.empty(2, dtype=torch.int32, device=device)
    abi.tmd_compute_forces_static(make_params(**params), n, float(box_length), _ptrs(p), _ptrs(f),
                                  int(ev.data_ptr()), int(st.data_ptr()), _stream())
    return f.t(), ev, st


class System:
    """Periodic cubic LJ box(es) advanced by the HIP library.

    ``System(n_atoms, box_length, **params)`` holds one box;
    ``System.batch(n_atoms, box_lengths, params)`` holds independent boxes
    advanced together in the same kernel launches.  Positions and velocities
    are float64 tensors of shape [N, 3] in original atom order (boxes
    concatenated).  All calls enqueue work on torch's current stream;
    ``sync()`` waits and raises on deferred device errors.
    """

    def __init__(self, n_atoms: int, box_length: float, device="cuda", _handle=None, _boxes=None, **params):
        abi.load_library()
        if _handle is None:
            self.params = [make_params(**params)]
            self.box_atoms = [int(n_atoms)]
            self.box_lengths = [float(box_length)]
            self._h = abi.tmd_create(self.params[0], self.box_atoms[0], self.box_lengths[0])
        else:
            self.params, self.box_atoms, self.box_lengths = _boxes
            self._h = _handle
        self.n = sum(self.box_atoms)
        self.nbox = len(self.box_atoms)
        _require_cuda()
        self.device = torch.device(device)
        nbytes = abi.tmd_workspace_size(self._h)
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-int(ws.data_ptr())) % 256
        self._ws = ws
        abi.tmd_bind_workspace(self._h, int(ws.data_ptr()) + off, nbytes)
        self._keep = []  # inputs kept alive until the next sync

    @classmethod
    def batch(cls, n_atoms: Sequence[int], box_lengths: Sequence[float], params=None, device="cuda"):
        """params: None (defaults), one dict for all boxes, or one dict per box."""
        nb = len(n_atoms)
        if params is None or isinstance(params, dict):
            plist = [make_params(**(params or {})) for _ in range(nb)]
        else:
            plist = [make_params(**p) for p in params]
        h = abi.tmd_create_batch(plist, [int(v) for v in n_atoms], [float(v) for v in box_lengths])
        return cls(0, 0.0, device=device, _handle=h,
                   _boxes=(plist, [int(v) for v in n_atoms], [float(v) for v in box_lengths]))

    # -- state -----------------------------------------------------------
    def set_state(self, pos, vel, step: int = 0) -> None:
        p = _soa(pos, self.n, self.device)
        v = _soa(vel, self.n, self.device)
        abi.tmd_set_state(self._h, _ptrs(p), _ptrs(v), int(step), _stream())
        self._keep = [p, v]

    def get_state(self):
        p = torch.empty(3, self.n, dtype=torch.float64, device=self.device)
        v = torch.empty(3, self.n, dtype=torch.float64, device=self.device)
        step = abi.tmd_get_state(self._h, _ptrs(p), _ptrs(v), _stream())
        return p.t(), v.t(), step

    # -- method ----------------------------------------------------------
    def build_neighbors(self) -> None:
        abi.tmd_build_neighbors(self._h, _stream())

    def compute_forces(self, energy: bool = True):
        """Returns (F [N,3], energy/virial or None): [U, W] for one box,
        [n_boxes, 2] for a batch."""
        f = torch.empty(3, self.n, dtype=torch.float64, device=self.device)
        ev = torch.empty(self.nbox, 2, dtype=torch.float64, device=self.device) if energy else None
        abi.tmd_compute_forces(self._h, _ptrs(f), int(ev.data_ptr()) if ev is not None else None, _stream())
        if ev is not None and self.nbox == 1:
            ev = ev[0]
        return f.t(), ev

    def integrate(self, n_steps: int, thermo_every: int = 0):
        """Advance n_steps; with thermo_every > 0 returns rows (KE, T, U, W, E):
        [n_steps // thermo_every, 5] for one box, [rows, n_boxes, 5] for a batch."""
        th = None
        rows = n_steps // thermo_every if thermo_every > 0 else 0
        if rows > 0:
            th = torch.empty(rows, self.nbox, 5, dtype=torch.float64, device=self.device)
        abi.tmd_integrate(self._h, int(n_steps), int(thermo_every) if rows > 0 else 0,
                          int(th.data_ptr()) if th is not None else None, _stream())
        if th is not None and self.nbox == 1:
            th = th[:, 0, :]
        return th

    def get_neighbors(self):
        """Returns (counts [N] int32, ids [N, max_neighbors] int32 sorted rows, -1 padded)."""
        m = self.params[0].max_neighbors
        counts = torch.empty(self.n, dtype=torch.int32, device=self.device)
        ids = torch.empty(self.n, m, dtype=torch.int32, device=self.device)
        abi.tmd_get_neighbors(self._h, int(counts.data_ptr()), int(ids.data_ptr()), self.n * m, _stream())
        return counts, ids

    def neighbor_counts(self):
        """List lengths [N] int32 in original atom order."""
        counts = torch.empty(self.n, dtype=torch.int32, device=self.device)
        abi.tmd_get_neighbors(self._h, int(counts.data_ptr()), None, 0, _stream())
        return counts

    def sync(self) -> None:
        abi.tmd_sync(self._h, _stream())
        self._keep = []

    def info(self) -> dict:
        return abi.tmd_get_info(self._h)

    def set_schedule(self, threads: int = 0, lds_atoms: int = 0, block_edge: int = 0, block_parts: int = 0,
                     lanes_per_atom: int = 0, build_threads: int = 0, build_lanes: int = 0) -> None:
        """Threads per force workgroup, LDS staging capacity, cells per block
        edge, workgroups per block, lanes per atom, threads per list-build
        workgroup and lanes per atom of the list build (0 = keep)."""
        abi.tmd_set_schedule(self._h, threads, lds_atoms, block_edge, block_parts, lanes_per_atom, build_threads,
                             build_lanes)

    LAYOUTS = {"soa": 0, "aos": 1, "aosoa": 2}

    def set_layout(self, layout) -> None:
        """Memory layout of the device positions: "soa", "aos" or "aosoa"
        (or 0, 1, 2); converts the current positions on the current stream."""
        code = self.LAYOUTS[layout] if isinstance(layout, str) else int(layout)
        abi.tmd_set_layout(self._h, code, _stream())

    def set_half_list(self, half: bool) -> None:
        """Half neighbor lists inside blocks (Newton's third law) for the
        Lennard-Jones model; needs one workgroup per block and one lane per
        atom.  The next step rebuilds the list."""
        abi.tmd_set_half_list(self._h, 1 if half else 0)

    def autotune(self, repeats: int = 5, cache: str | None = None, for_adjoint: bool = False):
        """Times each schedule (block edge, full or half lists, workgroups
        per block, lanes per atom, force and build threads, then the position
        layout) by one force evaluation plus a list build's share per step
        and keeps the fastest; returns a dict of block_edge, block_parts,
        lanes_per_atom, block_threads, build_threads, build_lanes, lds_atoms,
        half_list and layout, and "cached".  Rebuilds the list at the
        current positions.

        With ``cache`` (a JSON file path), a schedule stored there for the
        same device, library build and system shape is applied instead of
        tuning ("cached": True; the list is rebuilt at the next step), and
        a fresh pick is stored.  for_adjoint keeps to the schedules the
        adjoint runs with (full lists, SoA positions)."""
        key = None
        if cache is not None:
            key = tune_cache.system_key(torch.cuda.get_device_name(self.device), tune_cache.file_digest(abi.LIB_PATH),
                                        self.box_atoms, self.box_lengths, self.params, for_adjoint)
            hit = tune_cache.lookup(cache, key)
            if hit is not None:
                self.set_half_list(False)
                self.set_schedule(threads=hit["block_threads"], lds_atoms=hit["lds_atoms"],
                                  block_edge=hit["block_edge"], block_parts=hit["block_parts"],
                                  lanes_per_atom=hit["lanes_per_atom"], build_threads=hit["build_threads"],
                                  build_lanes=hit["build_lanes"])
                self.set_half_list(bool(hit["half_list"]))
                self.set_layout(hit["layout"])
                return dict(hit, cached=True)
        abi.tmd_autotune(self._h, repeats, _stream(), abi.TMD_TUNE_ADJOINT if for_adjoint else 0)
        info = self.info()
        sched = {k: info[k] for k in tune_cache.SCHEDULE_KEYS}
        if key is not None:
            tune_cache.store(cache, key, sched)
        return dict(sched, cached=False)

    def set_lj_params(self, epsilon, sigma) -> None:
        """Per-box epsilon and sigma (sequences of n_boxes floats, or scalars)."""
        eps = [float(epsilon)] * self.nbox if isinstance(epsilon, (int, float)) else [float(v) for v in epsilon]
        sig = [float(sigma)] * self.nbox if isinstance(sigma, (int, float)) else [float(v) for v in sigma]
        abi.tmd_set_lj_params(self._h, eps, sig, _stream())
        for p, e, s in zip(self.params, eps, sig):
            p.epsilon, p.sigma = e, s

    def adjoint_forward(self, n_steps: int) -> None:
        """Integrate n_steps, recording checkpoints for adjoint_backward()."""
        nbytes = abi.tmd_adjoint_workspace_size(self._h, int(n_steps))
        if getattr(self, "_adj_ws", None) is None or self._adj_ws.numel() < nbytes + 256:
            self._adj_ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        self._adj_ptr = int(self._adj_ws.data_ptr()) + (-int(self._adj_ws.data_ptr())) % 256
        self._adj_bytes = nbytes
        abi.tmd_adjoint_forward(self._h, int(n_steps), self._adj_ptr, nbytes, _stream())

    def adjoint_backward(self, lam_x, lam_v=None):
        """Cotangents of the final (x, v) -> (dL/dx0 [N,3], dL/dv0 [N,3],
        dL/deps [n_boxes], dL/dsigma [n_boxes])."""
        lx = _soa(lam_x, self.n, self.device)
        lv = _soa(lam_v, self.n, self.device) if lam_v is not None else None
        gx = torch.empty(3, self.n, dtype=torch.float64, device=self.device)
        gv = torch.empty(3, self.n, dtype=torch.float64, device=self.device)
        ge = torch.empty(self.nbox, dtype=torch.float64, device=self.device)
        gs = torch.empty(self.nbox, dtype=torch.float64, device=self.device)
        abi.tmd_adjoint_backward(self._h, self._adj_ptr, self._adj_bytes, _ptrs(lx),
                                 _ptrs(lv) if lv is not None else None, _ptrs(gx), _ptrs(gv), int(ge.data_ptr()),
                                 int(gs.data_ptr()), _stream())
        self._keep = [lx, lv]
        return gx.t(), gv.t(), ge, gs

    def set_graphs(self, enable: bool) -> None:
        """Run whole rebuild intervals of integrate() as captured HIP graphs
        (bit-identical results; see tmd_set_graphs)."""
        abi.tmd_set_graphs(self._h, enable)

    def set_timing(self, enable: bool) -> None:
        abi.tmd_set_timing(self._h, enable)

    def get_timing(self) -> dict:
        return abi.tmd_get_timing(self._h)

    def close(self) -> None:
        if getattr(self, "_h", None):
            try:
                torch.cuda.synchronize(self.device)
            finally:
                abi.tmd_destroy(self._h)
                self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
