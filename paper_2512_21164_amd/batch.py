"""Batched execution of many GADI systems (C-ABI gadi_batch_*).

Each member is a ``Solver`` (its own workspace and Krylov state).  One
``step(n)`` advances every unfinished member by n phases of its own state
machine, in one captured graph of persistent step launches per kernel
class; members are independent (each keeps its own reductions, so a
member's result does not depend on the rest of the batch).
"""
from __future__ import annotations

import ctypes as C

from . import _lib
from .api import _stream_handle


class Batch:
    def __init__(self, max_systems: int, stream=None, device="cuda"):
        import torch
        self.lib = _lib.load()
        self.max_systems = int(max_systems)
        nb = C.c_size_t(0)
        _lib.check(self.lib.gadi_batch_workspace_bytes(self.max_systems, C.byref(nb)), "gadi_batch_workspace_bytes")
        self.workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=device)
        self.stream = stream
        self.handle = C.c_void_p()
        _lib.check(self.lib.gadi_batch_create(self.max_systems, C.c_void_p(_stream_handle(stream)),
                                              C.c_void_p(self.workspace.data_ptr()), nb, C.byref(self.handle)),
                   "gadi_batch_create")
        self.members = {}

    def add(self, solver, b, x) -> int:
        """Start solving A x = b with ``solver`` inside the batch; returns the slot."""
        solver._check_vec(b)
        solver._check_vec(x)
        slot = C.c_int32(-1)
        _lib.check(self.lib.gadi_batch_add(self.handle, solver.handle, C.c_void_p(b.data_ptr()),
                                           C.c_void_p(x.data_ptr()), C.byref(slot)), "gadi_batch_add")
        self.members[slot.value] = (solver, b, x)
        return slot.value

    def step(self, nsteps: int):
        _lib.check(self.lib.gadi_batch_step(self.handle, int(nsteps)), "gadi_batch_step")

    def poll(self):
        """Synchronize; returns (list of finished slots, number still active)."""
        done = (C.c_int32 * self.max_systems)()
        active = C.c_int32(0)
        _lib.check(self.lib.gadi_batch_poll(self.handle, done, C.byref(active)), "gadi_batch_poll")
        return [i for i in range(self.max_systems) if done[i] and i in self.members], active.value

    def remove(self, slot: int):
        """Report of a finished member; the member leaves the batch. Returns (solver, b, x, report)."""
        rep = _lib.gadi_report()
        st = _lib.check(self.lib.gadi_batch_remove(self.handle, int(slot), C.byref(rep), None), "gadi_batch_remove")
        out = rep.as_dict()
        out["status_name"] = self.lib.gadi_status_string(st).decode()
        solver, b, x = self.members.pop(slot)
        return solver, b, x, out

    def run(self, steps_per_launch: int = 32):
        """Run until every member has finished; returns {slot: report}."""
        reports = {}
        while self.members:
            self.step(steps_per_launch)
            done, _ = self.poll()
            for s in done:
                reports[s] = self.remove(s)[3]
        return reports

    def close(self):
        if self.handle:
            self.lib.gadi_batch_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
