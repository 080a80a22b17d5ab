"""Python front end of one periodic LJ box on one GPU.

PyTorch provides device memory (the library's workspace and the caller's
arrays) and the stream (torch's current stream); every step of the method
runs in the HIP library through the C ABI in ``_abi``.
"""

from __future__ import annotations

import torch

from . import _abi as abi


def _stream() -> int:
    return int(torch.cuda.current_stream().cuda_stream)


def _require_cuda():
    if not torch.cuda.is_available():
        raise RuntimeError("paper_2009_07400_amd needs a ROCm GPU (torch.cuda.is_available() is False)")


def _soa(t: torch.Tensor, n: int, device) -> torch.Tensor:
    """[N,3] or [3,N] -> contiguous float64 [3,N] on the device."""
    t = torch.as_tensor(t, dtype=torch.float64, device=device)
    if t.shape == (n, 3):
        t = t.t()
    if t.shape != (3, n):
        raise ValueError(f"expected shape ({n}, 3) or (3, {n}), got {tuple(t.shape)}")
    return t.contiguous()


def _ptrs(t3: torch.Tensor):
    return [int(t3[k].data_ptr()) for k in range(3)]


def make_params(epsilon=1.0, sigma=1.0, mass=1.0, cutoff=2.5, skin=0.3, dt=0.005, rebuild_every=20,
                max_neighbors=128) -> abi.TmdParams:
    return abi.TmdParams(epsilon, sigma, mass, cutoff, skin, dt, rebuild_every, max_neighbors)


class System:
    """A periodic cubic LJ box advanced by the HIP library.

    Positions and velocities are exchanged as float64 tensors of shape [N, 3]
    in original atom order.  All calls enqueue work on torch's current stream;
    ``sync()`` waits and raises on deferred device errors.
    """

    def __init__(self, n_atoms: int, box_length: float, device="cuda", **params):
        abi.load_library()
        self.params = make_params(**params)
        self.n = int(n_atoms)
        self.box_length = float(box_length)
        self._h = abi.tmd_create(self.params, self.n, self.box_length)
        _require_cuda()
        self.device = torch.device(device)
        nbytes = abi.tmd_workspace_size(self._h)
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-int(ws.data_ptr())) % 256
        self._ws = ws
        abi.tmd_bind_workspace(self._h, int(ws.data_ptr()) + off, nbytes)
        self._keep = []  # inputs kept alive until the next sync

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
        """Returns (F [N,3], tensor([U, W]) or None)."""
        f = torch.empty(3, self.n, dtype=torch.float64, device=self.device)
        ev = torch.empty(2, dtype=torch.float64, device=self.device) if energy else None
        abi.tmd_compute_forces(self._h, _ptrs(f), int(ev.data_ptr()) if ev is not None else None, _stream())
        return f.t(), ev

    def integrate(self, n_steps: int, thermo_every: int = 0):
        """Advance n_steps; returns thermo rows [n_steps // thermo_every, 5]
        (KE, T, U, W, E) when thermo_every > 0, else None."""
        th = None
        rows = n_steps // thermo_every if thermo_every > 0 else 0
        if rows > 0:
            th = torch.empty(rows, 5, dtype=torch.float64, device=self.device)
        abi.tmd_integrate(self._h, int(n_steps), int(thermo_every) if rows > 0 else 0,
                          int(th.data_ptr()) if th is not None else None, _stream())
        return th

    def get_neighbors(self):
        """Returns (counts [N] int32, ids [N, max_neighbors] int32 sorted rows, -1 padded)."""
        m = self.params.max_neighbors
        counts = torch.empty(self.n, dtype=torch.int32, device=self.device)
        ids = torch.empty(self.n, m, dtype=torch.int32, device=self.device)
        abi.tmd_get_neighbors(self._h, int(counts.data_ptr()), int(ids.data_ptr()), self.n * m, _stream())
        return counts, ids

    def sync(self) -> None:
        abi.tmd_sync(self._h, _stream())
        self._keep = []

    def info(self) -> dict:
        return abi.tmd_get_info(self._h)

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
