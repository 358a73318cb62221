"""Learned student NEP: teacher-labelled bead snapshots, training, judged use.

A smaller NEP (the student) stands in for the full model (the teacher)
inside the PIMD loop:

1. `teacher_snapshots` runs teacher NEP-PIMD (Sec. II.A driver, Sec. II.C
   model) at one or more temperatures and keeps every `every`-th step's bead
   positions with the teacher's energies, forces and virials, all resident
   in device memory (`SnapshotStore`).
2. `StudentTrainer` fits the student to those labels with the library's
   training kernels (loss on energy, force and virial residuals; gradient
   by a forward-mode descriptor pass; Adam), holding out a share of the
   snapshots for validation.
3. `StudentPimd` integrates with student forces (network on the matrix
   cores) and lets the teacher judge them every `judge_every` steps on the
   same positions; when the force RMSE exceeds the threshold the teacher
   takes over for the rest of the run.

The paper fits its NEP models by evolutionary search (SNES); gradient
training of a student is this library's addition.
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Optional, Sequence

import numpy as np

from . import inputs as I
from . import lib
from .engine import NepPimd, default_capacity


class SnapshotStore:
    """Bead snapshots of one system, resident on the device.

    pos [C,P,N,3] f64, E [C,P] f64, F [C,P,N,3] f32, W [C,P,9] f64, T [C]."""

    def __init__(self, capacity: int, P: int, N: int):
        import torch
        dev = torch.device("cuda")
        self.capacity, self.P, self.N = int(capacity), int(P), int(N)
        self.pos = torch.empty((capacity, P, N, 3), dtype=torch.float64, device=dev)
        self.E = torch.empty((capacity, P), dtype=torch.float64, device=dev)
        self.F = torch.empty((capacity, P, N, 3), dtype=torch.float32, device=dev)
        self.W = torch.empty((capacity, P, 9), dtype=torch.float64, device=dev)
        self.T = np.zeros(capacity)
        self.n = 0

    def __len__(self):
        return self.n

    def add(self, pos, E, F, W, T: float):
        if self.n >= self.capacity:
            raise ValueError(f"snapshot store is full ({self.capacity})")
        k = self.n
        self.pos[k].copy_(pos)
        self.E[k].copy_(E)
        self.F[k].copy_(F)
        self.W[k].copy_(W)
        self.T[k] = T
        self.n += 1

    def bead_snapshots(self) -> int:
        return self.n * self.P


def teacher_snapshots(teacher_path: str, make_system, temperatures: Sequence[float], *, steps: int, every: int,
                      warmup: int, dt: float, mode: str = "trpmd", tau: float = 100.0, seed: int = 0,
                      store: Optional[SnapshotStore] = None, skin: float = 0.5, check_every: int = 50,
                      prepare=None) -> SnapshotStore:
    """Teacher NEP-PIMD at each temperature; keep every `every`-th step after `warmup`.

    make_system(T) returns the starting `inputs.System` (P beads) at T.  A
    kept snapshot is the positions at which the step evaluated its forces,
    with the teacher's E [P], F [P,N,3] and W [P,9] there.  Snapshots of a
    poll window are staged and enter the store only once the engine's poll
    at the end of the window has verified the lists; a window replayed after
    a row overflow records its snapshots again from the replay.  prepare(eng),
    if given, is applied to each engine before its first step."""
    per_T = (steps + every - 1) // every
    for k, T in enumerate(temperatures):
        system = make_system(T)
        if store is None:
            store = SnapshotStore(per_T * len(temperatures), system.P, system.N)
        eng = NepPimd(teacher_path, system, dt=dt, T=T, tau=tau, mode=mode, seed=seed + 7919 * k,
                      check_every=0, skin=skin)
        pending: list = []
        committed = [0]

        def record(n, eng=eng, pending=pending):
            if n >= warmup and (n - warmup) % every == 0:
                pending.append((eng.pos.clone(), eng.E.clone(), eng.F.clone(), eng.W.clone()))

        def save(pending=pending, committed=committed):
            return committed[0] + len(pending)

        def restore(tok, pending=pending, committed=committed):
            del pending[tok - committed[0]:]

        def commit(T=T, pending=pending, committed=committed):
            for x, E, F, W in pending:
                store.add(x, E, F, W, T)
            committed[0] += len(pending)
            pending.clear()

        eng.on_forces = record
        eng.snapshot_hooks.append((save, restore))
        if prepare is not None:
            prepare(eng)
        eng._snapshot()
        eng.start()
        for s in range(warmup + steps):
            eng.step()
            if (s + 1) % check_every == 0:
                eng.check()
                commit()
        eng.check()
        commit()
    return store


@dataclasses.dataclass
class TrainLog:
    epoch: int
    lr: float
    loss: float
    val_rmse_F: float     # eV/A
    seconds: float


class StudentTrainer:
    """Fits a student model to teacher-labelled snapshots on the device."""

    def __init__(self, student_path: str, store: SnapshotStore, types, box, *, lambdas=(1.0, 1.0, 0.1),
                 holdout: float = 0.1, seed: int = 0, mask: int = 7, skin: float = 0.5):
        import torch
        self.torch = torch
        self.store = store
        self.model = lib.Model(student_path)
        self.P, self.N = store.P, store.N
        self.box = np.asarray(box, np.float64)
        self.types = torch.as_tensor(np.asarray(types), dtype=torch.int32, device="cuda").contiguous()
        self.lambdas = tuple(float(x) for x in lambdas)
        self.mask = mask
        rng = np.random.default_rng(seed)
        order = rng.permutation(len(store))
        n_val = max(1, int(round(holdout * len(store)))) if len(store) > 1 else 0
        self.val = np.sort(order[:n_val])
        self.train = np.sort(order[n_val:]) if n_val < len(store) else order
        self.rng = rng
        dens = self.N / I.cell_volume(self.box)
        caps = (default_capacity(self.model.rc_radial + skin + 1.0, dens, 1),
                default_capacity(self.model.rc_angular + skin + 1.0, dens, 1))
        self.nl = lib.fitted_neighbor_list(self.model, store.pos[0], self.box, self.types, *caps, skin=skin)
        self.ws = lib.Workspace(self.model, self.P, self.N)
        self.trainer = lib.Trainer(self.model, self.P, self.N)
        self.skin = skin
        self._groups = {}   # snapshots per call -> (lists, workspace, trainer, types) of that batch
        self.E = torch.zeros(self.P, dtype=torch.float64, device="cuda")
        self.F = torch.zeros((self.P, self.N, 3), dtype=torch.float32, device="cuda")
        self.W = torch.zeros((self.P, 9), dtype=torch.float64, device="cuda")
        self.work = torch.empty(1025, dtype=torch.float64, device="cuda")
        self.log: List[TrainLog] = []

    def _check_lists(self):
        st = self.nl.status(clear=True)
        if st["flags"] & lib.FLAG_NEIGHBOR_OVERFLOW:
            raise lib.NepError(5, "student training: candidate rows overflowed")
        if st["flags"] or self.ws.poll(clear=True):
            raise lib.NepError(6, f"student training: device flags {st['flags']:#x}")

    def _group(self, B: int):
        """Handles for B snapshots per gradient call (a batch of B systems of N atoms)."""
        g = self._groups.get(B)
        if g is None:
            off = np.arange(B + 1, dtype=np.int32) * self.N
            nl = lib.NeighborList(self.model, self.P, B * self.N, *self.nl.caps, offsets=off)
            nl.set_skin(self.skin)
            ws = lib.Workspace(self.model, self.P, B * self.N, offsets=off)
            tr = lib.Trainer(self.model, self.P, B * self.N, sys_offsets=off, share=self.trainer)
            g = (nl, ws, tr, self.types.repeat(B).contiguous(), np.stack([self.box] * B))
            self._groups[B] = g
        return g

    def _check_groups(self):
        for nl, ws, _, _, _ in self._groups.values():
            st = nl.status(clear=True)
            if st["flags"] & lib.FLAG_NEIGHBOR_OVERFLOW:
                raise lib.NepError(5, "student training: candidate rows overflowed")
            if st["flags"] or ws.poll(clear=True):
                raise lib.NepError(6, f"student training: device flags {st['flags']:#x}")

    def epoch(self, lr: float, batch: int = 1) -> float:
        """One pass over the training snapshots in random order; one gradient call
        (the snapshots as a batch of systems) and one Adam step per `batch`
        snapshots.  Returns the mean loss per snapshot."""
        t = self.torch
        st = self.store
        idx = self.rng.permutation(self.train)
        total = t.zeros(4, dtype=t.float64, device="cuda")
        P, N = self.P, self.N
        for s in range(0, len(idx), batch):
            ks = idx[s:s + batch]
            self.trainer.zero()
            if len(ks) == 1:
                k = int(ks[0])
                self.nl.build(st.pos[k], self.box, self.types)
                self.trainer.accumulate(self.nl, self.ws, st.pos[k], self.box, self.types, st.E[k], st.F[k],
                                        st.W[k], self.lambdas)
            else:
                B = len(ks)
                nl, ws, tr, types, boxes = self._group(B)
                sel = t.as_tensor(ks, device="cuda")
                # [B, P, N, 3] -> [P, B N, 3]: the snapshots side by side along the atom axis
                pos = st.pos.index_select(0, sel).permute(1, 0, 2, 3).reshape(P, B * N, 3).contiguous()
                F = st.F.index_select(0, sel).permute(1, 0, 2, 3).reshape(P, B * N, 3).contiguous()
                nl.build(pos, boxes, types)
                tr.accumulate(nl, ws, pos, boxes, types, st.E.index_select(0, sel).contiguous(), F,
                              st.W.index_select(0, sel).contiguous(), self.lambdas)
            total += self.trainer.loss
            self.trainer.adam(lr, mask=self.mask)
        self._check_lists()
        self._check_groups()
        return float(total[0]) / max(1, len(idx))

    def rmse(self, which: str = "val") -> float:
        """Force RMSE (eV/A, over every component) of the current student against the teacher labels."""
        t = self.torch
        st = self.store
        idx = self.val if which == "val" else self.train
        if len(idx) == 0:
            return float("nan")
        acc = t.zeros((), dtype=t.float64, device="cuda")
        for k in idx:
            self.nl.build(st.pos[k], self.box, self.types)
            self.ws.compute(self.nl, st.pos[k], self.box, self.types, self.E, self.F, self.W)
            r = lib.force_rmse(self.F, st.F[k], self.work)
            acc += r * r
        self._check_lists()
        return float(t.sqrt(acc / len(idx)))

    def fit(self, epochs: int, lr0: float = 5e-3, lr1: float = 2e-4, batch: int = 1, time_budget: float = None,
            every: int = 1, verbose: bool = False) -> List[TrainLog]:
        """Exponentially decaying learning rate lr0 -> lr1 over `epochs` (or the time budget, seconds)."""
        t0 = time.perf_counter()
        for e in range(epochs):
            lr = lr0 * (lr1 / lr0) ** (e / max(1, epochs - 1))
            loss = self.epoch(lr, batch)
            if (e + 1) % every == 0 or e == epochs - 1:
                r = self.rmse("val")
                self.log.append(TrainLog(e + 1, lr, loss, r, time.perf_counter() - t0))
                if verbose:
                    print(f"[student] epoch {e + 1}: lr {lr:.2e} loss {loss:.4e} val force RMSE {1e3 * r:.2f} meV/A",
                          flush=True)
            if time_budget is not None and time.perf_counter() - t0 > time_budget:
                break
        return self.log

    def save(self, path: str):
        I.write_model(path, self.model.to_dict())


class StudentPimd:
    """NEP-PIMD on student forces, judged by the teacher every `judge_every` steps.

    At a judge step the teacher evaluates the same bead positions on the
    same neighbour lists (teacher and student share their cutoffs); the
    force RMSE over all beads, atoms and components decides: above
    `threshold` (eV/A) the teacher's forces are used for that step and every
    later one (fallback), otherwise the student continues.  `history` keeps
    (step, RMSE) of every judgement."""

    def __init__(self, teacher_path: str, student_path: str, system, *, dt: float, T: float, tau: float = 100.0,
                 mode: str = "trpmd", seed: int = 0, judge_every: int = 50, threshold: float = 0.020,
                 mlp: int = lib.MLP_BF16_MFMA, check_every: int = 50, skin: float = 0.5):
        import torch
        self.torch = torch
        self.eng = NepPimd(student_path, system, dt=dt, T=T, tau=tau, mode=mode, seed=seed, check_every=0,
                           skin=skin)
        if mlp != lib.MLP_FP32:
            self.eng.model.set_mlp(mlp)
        self.teacher = lib.Model(teacher_path)
        sm = self.eng.model
        if (self.teacher.rc_radial, self.teacher.rc_angular) != (sm.rc_radial, sm.rc_angular) or \
                self.teacher.n_species != sm.n_species:
            raise ValueError("teacher and student must share cutoffs and species (one set of lists)")
        e = self.eng
        self.tws = lib.Workspace(self.teacher, e.P, e.N)
        self.Et = torch.zeros_like(e.E)
        self.Ft = torch.zeros_like(e.F)
        self.Wt = torch.zeros_like(e.W)
        self.work = torch.empty(1025, dtype=torch.float64, device="cuda")
        self.judge_every = int(judge_every)
        self.threshold = float(threshold)
        self.check_every = check_every
        self.on_student = True
        self.fallback_step: Optional[int] = None
        self.history: List[tuple] = []
        # a replay after a row overflow goes through the judged step, and the
        # judge's state rolls back with the engine's snapshot
        e.replay_step = self._advance
        e.snapshot_hooks.append((self._save, self._restore))
        e._snapshot()

    def _save(self):
        return (self.on_student, self.fallback_step, len(self.history))

    def _restore(self, tok):
        self.on_student, self.fallback_step, n = tok
        del self.history[n:]
        # flags the teacher raised in the discarded window (forces on
        # truncated rows) do not outlive it; the replay raises its own
        self.tws.poll(clear=True)

    @property
    def step_no(self):
        return self.eng.step_no

    def _teacher(self, E, F, W):
        e = self.eng
        self.tws.compute(e.nl, e.pos, e.box, e.types, E, F, W)

    def forces(self, judge: bool = True):
        e = self.eng
        e.nl.build(e.pos, e.box, e.types)
        if not self.on_student:
            self._teacher(e.E, e.F, e.W)
            return
        e.ws.compute(e.nl, e.pos, e.box, e.types, e.E, e.F, e.W)
        if judge and self.judge_every and e.step_no % self.judge_every == 0:
            self._teacher(self.Et, self.Ft, self.Wt)
            r = float(lib.force_rmse(e.F, self.Ft, self.work))
            self.history.append((e.step_no, r))
            if not r <= self.threshold:
                # the teacher's forces at these positions drive this step and the rest of the run
                self.on_student = False
                self.fallback_step = e.step_no
                e.E, self.Et = self.Et, e.E
                e.F, self.Ft = self.Ft, e.F
                e.W, self.Wt = self.Wt, e.W

    def start(self):
        e = self.eng
        self.forces(judge=False)
        e.pimd.step(e.pos, e.vel, e.F, e.step_no, lib.PRE)
        e.started = True

    def check(self):
        """Poll the lists and both workspaces (synchronises); raise on device flags."""
        self.eng.check()
        if self.tws.poll(clear=True):
            raise lib.NepError(6, "teacher evaluation raised device flags")

    def _advance(self):
        """One judged step without a poll (also the engine's replay step)."""
        e = self.eng
        if not e.started:
            self.start()
        self.forces()
        e.pimd.step(e.pos, e.vel, e.F, e.step_no, lib.FUSED)
        e.step_no += 1

    def step(self):
        self._advance()
        if self.check_every and self.eng.step_no % self.check_every == 0:
            self.check()

    def run(self, n: int):
        for _ in range(n):
            self.step()
