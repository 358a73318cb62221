"""Driver loop of the hot path: neighbour build -> NEP forces -> integrator.

One stream, no per-step host synchronisation: the sticky device flags of
the neighbour lists and of the force workspace are polled every
`check_every` steps.  Each successful poll keeps a device snapshot of the
state; a candidate-row overflow found by a poll grows the rows, rolls back
to the snapshot and replays the steps (the noise is counter-based, so the
replay is the trajectory that larger rows would have given).  Regrowth is
bounded: at most `max_regrow` rounds and `regrow_budget_s` seconds per poll,
after which the poll raises with the capacities and the step reached.  The
step is the paper's workflow (Sec. II.A): thermostat,
half kick, free ring-polymer step, forces, half kick, thermostat; the two
integrator halves around consecutive force evaluations run as one fused
launch.  Optional: the ring-polymer observables (centroid virial kinetic
energy, virial and pressure tensors) recorded on the device after the
closing half of every k-th step, a Berendsen-like barostat after the
closing half of every step (Sec. II.D), and centroid velocities dumped
every k-th step (these split the fused launch); partial radial
distribution functions accumulated on the device from the neighbour lists
of every k-th force call.
"""
from __future__ import annotations

import math
import time
from typing import Callable, List, Optional

import numpy as np

from . import inputs as I
from . import lib


def default_capacity(rc: float, density: float, n_species: int, slack: float = 1.6) -> int:
    """First guess of a candidate row length from the mean density (refitted after one build)."""
    n = density * 4.0 / 3.0 * math.pi * rc ** 3
    return int(math.ceil(n * slack)) + 8


def rdf_normalise(counts, n_per_species, volume: float, rmax: float, frames: int, P: int):
    """g_ab(r_k) = counts_ab[k] / (frames P N_a rho_b V_k), rho_b = (N_b - [a == b]) / V,
    V_k the volume of shell k of width rmax / nbins; bins of an absent species are 0."""
    c = np.asarray(counts, np.float64)
    S, nb = c.shape[0], c.shape[2]
    edges = np.linspace(0.0, rmax, nb + 1)
    shell = (4.0 * np.pi / 3.0) * np.diff(edges ** 3)
    g = np.zeros_like(c)
    for a in range(S):
        for b in range(S):
            pairs = n_per_species[a] * (n_per_species[b] - (a == b))
            if pairs > 0 and frames > 0:
                g[a, b] = c[a, b] * volume / (frames * P * pairs * shell)
    return 0.5 * (edges[1:] + edges[:-1]), g


class NepPimd:
    """NEP forces for P beads of one periodic system, or of a batch of
    independent systems of uneven size, plus the ring-polymer integrator.

    With a list of systems the atoms are concatenated along the atom axis,
    every kernel of a step covers all systems at once, and E / W gain a
    leading system axis ([nsys, P], [nsys, P, 9]).

    mlp selects the network arithmetic: "auto" (FP32 accuracy, matrix cores
    or vector units by the model's shape), "fp32", "fp32_mfma" or
    "bf16_mfma"; self.mlp is the arithmetic in use."""

    def __init__(self, model_path: str, system, *, dt: float, T: float, tau: float = 100.0,
                 mode: str = "trpmd", seed: int = 0, caps: Optional[tuple] = None, check_every: int = 50,
                 want_atom: bool = False, skin: float = 0.5, autotune: bool = False, obs_every: int = 0,
                 barostat: Optional[dict] = None, rdf: Optional[dict] = None, dump_every: int = 0,
                 max_regrow: int = 8, regrow_budget_s: float = 300.0, d3: Optional[str] = None,
                 mlp: str = "auto"):
        import torch
        self.torch = torch
        dev = torch.device("cuda")
        self.model = lib.Model(model_path)
        if mlp not in lib.MLP_MODES:
            raise ValueError(f"mlp must be one of {sorted(lib.MLP_MODES)}")
        if lib.MLP_MODES[mlp] != lib.MLP_FP32:
            self.model.set_mlp(lib.MLP_MODES[mlp])
        self.mlp = lib.MLP_NAMES[self.model.mlp]   # "auto" resolved by the library
        systems = list(system) if isinstance(system, (list, tuple)) else [system]
        self.batched = isinstance(system, (list, tuple))
        self.P = systems[0].P
        if any(s.P != self.P for s in systems):
            raise ValueError("all systems of a batch need the same number of beads")
        sizes = [s.N for s in systems]
        self.offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
        self.N = int(self.offsets[-1])
        self.nsys = len(systems)
        self.box = np.stack([np.asarray(s.box, np.float64) for s in systems]) if self.batched \
            else np.asarray(systems[0].box, np.float64)
        cat = lambda f, ax: np.concatenate([f(s) for s in systems], axis=ax)
        self.pos = torch.tensor(cat(lambda s: s.pos, 1), dtype=torch.float64, device=dev)
        self.vel = torch.tensor(cat(lambda s: s.vel, 1), dtype=torch.float64, device=dev)
        self.types = torch.tensor(cat(lambda s: s.types, 0), dtype=torch.int32, device=dev)
        self.mass = torch.tensor(cat(lambda s: s.masses, 0), dtype=torch.float64, device=dev)
        self.F = torch.zeros((self.P, self.N, 3), dtype=torch.float32, device=dev)
        eshape = (self.nsys, self.P) if self.batched else (self.P,)
        self.E = torch.zeros(eshape, dtype=torch.float64, device=dev)
        self.W = torch.zeros(eshape + (9,), dtype=torch.float64, device=dev)
        self.E_atom = torch.zeros((self.P, self.N), dtype=torch.float32, device=dev) if want_atom else None
        self.W_atom = torch.zeros((self.P, self.N, 9), dtype=torch.float32, device=dev) if want_atom else None
        vol = sum(I.cell_volume(s.box) for s in systems)
        dens = self.N / vol
        self.density = dens
        S = self.model.n_species
        rcR, rcA = self.model.rc_radial, self.model.rc_angular
        self.caps = tuple(caps) if caps else (default_capacity(rcR + 0.5 + skin, dens, S),
                                              default_capacity(rcA + 0.5 + skin, dens, S))
        self.nl = None
        self.skin = skin
        offs = self.offsets if self.batched else None
        self.ws = lib.Workspace(self.model, self.P, self.N, offsets=offs)
        self.pimd = lib.Pimd(self.P, self.N, self.mass, dt, T, tau, mode, seed)
        self.check_every = check_every
        self.step_no = 0
        self.started = False
        self.graph = None
        self.graph_steps = 0
        self.step_dev = None      # two alternating device step counters of the captured steps
        self._dev_stale = False   # an eager step ran since the last replay: refresh the counter first
        self.obs_every = int(obs_every)
        self.baro = dict(barostat) if barostat else None
        self.obs_log = []
        if (self.obs_every or self.baro) and self.batched:
            raise ValueError("observables and the barostat need a single system")
        self.obs = torch.zeros(lib.OBS_COUNT, dtype=torch.float64, device=dev)
        self.mu = torch.ones(3, dtype=torch.float64, device=dev)
        # partial RDFs: rdf = dict(rmax=A, nbins=n, every=k)
        self.rdf_cfg = dict(rdf) if rdf else None
        self.rdf_frames = 0
        self.rdf_hist = None
        if self.rdf_cfg:
            if self.batched:
                raise ValueError("the radial distribution functions need a single system")
            S_ = self.model.n_species
            self.rdf_hist = torch.zeros((S_, S_, int(self.rdf_cfg["nbins"])), dtype=torch.int64, device=dev)
        self.dump_every = int(dump_every)
        self.dump_log = []
        if self.dump_every and self.batched:
            raise ValueError("velocity dumps need a single system")
        # D3 dispersion (NEP-D3): its own lists (dispersion / coordination cutoffs) on the same positions
        self.d3 = lib.D3(d3) if d3 else None
        self.d3_nl = None
        self.d3_caps = None
        if self.d3 is not None:
            if self.batched:
                raise ValueError("the D3 term needs a single system")
            if self.d3.n_species != self.model.n_species:
                raise ValueError("the D3 parameters and the model have different species counts")
            self.d3_ws = self.d3.workspace(self.P, self.N)
        self.rollbacks = 0
        self.rebuilds_total = 0      # candidate-row rebuilds counted by the successful polls
        self.max_regrow = int(max_regrow)
        self.regrow_budget_s = float(regrow_budget_s)
        # Owners of extra per-step state (a student driver, snapshot recording):
        # on_forces(n) runs after the forces of step n (eager steps, replays
        # included); snapshot_hooks are (save() -> token, restore(token)) pairs
        # taken with every device snapshot and restored on a rollback;
        # replay_step, if set, replays one step instead of self.step.
        self.on_forces: Optional[Callable[[int], None]] = None
        self.snapshot_hooks: List[tuple] = []
        self.replay_step: Optional[Callable[[], None]] = None
        self._snap = None
        self._finished = False   # the last call was finish() (closing half without the next opening half)
        self._fit_capacity()
        self._snapshot()
        self.tile = None   # autotuned (waves per group, weight staging, {(waves, staging): ms})
        if autotune:
            self.tile = self.ws.autotune(self.nl, self.pos, self.box, self.types, self.E, self.F, self.W)

    # ------------------------------------------------------------------
    def _fit_capacity(self):
        """Size the candidate rows to the starting configuration, with room for
        the ring polymers to spread: the rows are at least as long as a uniform
        system of the same density needs for radius rc + skin + 2 A (the ring
        polymers spread and the local density fluctuates during a run; a row
        that still overflows is grown by `check`)."""
        self.nl = lib.fitted_neighbor_list(self.model, self.pos, self.box, self.types, *self.caps, skin=self.skin,
                                           offsets=self.offsets if self.batched else None)
        floor = (default_capacity(self.model.rc_radial + self.skin + 2.0, self.density, 1, slack=1.3),
                 default_capacity(self.model.rc_angular + self.skin + 2.0, self.density, 1, slack=1.3))
        caps = tuple(max(a, b) for a, b in zip(self.nl.caps, floor))
        if caps != tuple(self.nl.caps):
            self.nl = lib.NeighborList(self.model, self.P, self.N, *caps,
                                       offsets=self.offsets if self.batched else None)
            self.nl.set_skin(self.skin)
            self.nl.build(self.pos, self.box, self.types)
        self.caps = caps
        if self.d3 is not None:
            lm = self.d3.list_model
            guess = (default_capacity(lm.rc_radial + self.skin + 1.0, self.density, 1),
                     default_capacity(lm.rc_angular + self.skin + 1.0, self.density, 1))
            self.d3_nl = lib.fitted_neighbor_list(lm, self.pos, self.box, self.types, *guess, skin=self.skin)
            floor = (default_capacity(lm.rc_radial + self.skin + 2.0, self.density, 1, slack=1.3),
                     default_capacity(lm.rc_angular + self.skin + 2.0, self.density, 1, slack=1.3))
            d3c = tuple(max(a, b) for a, b in zip(self.d3_nl.caps, floor))
            if d3c != tuple(self.d3_nl.caps):
                self.d3_nl = self._d3_list(d3c)
            self.d3_caps = d3c

    def _d3_list(self, caps):
        nl = lib.NeighborList(self.d3.list_model, self.P, self.N, *caps)
        nl.set_skin(self.skin)
        nl.build(self.pos, self.box, self.types)
        return nl

    def _fold(self) -> bool:
        """Whether a step may leave the per-bead E/W sums to its integrator
        launch: nothing reads E or W between the forces and the stage (no D3
        term accumulating into them, no force hook, no observables)."""
        return self.d3 is None and self.on_forces is None and not self._split()

    def forces(self, defer: bool = False):
        """Neighbour lists + NEP energy, forces and virial at the current positions
        (plus the D3 dispersion term when the engine has one).  defer: E and W
        are completed by the next `pimd.step_nep` with this workspace."""
        self.nl.build(self.pos, self.box, self.types)
        if defer:
            self.ws.defer_reduce()
        self.ws.compute(self.nl, self.pos, self.box, self.types, self.E, self.F, self.W, self.E_atom, self.W_atom)
        if self.d3 is not None:
            self.d3_nl.build(self.pos, self.box, self.types)
            self.d3.compute(self.d3_nl, self.d3_ws, self.pos, self.box, self.types, self.E, self.F, self.W,
                            accumulate=True)

    def check(self):
        """Poll the sticky flags (synchronises).  A candidate-row overflow since
        the last poll grows the rows, rolls back to the last poll's snapshot and
        replays the steps, at most `max_regrow` times and for at most
        `regrow_budget_s` seconds; non-finite values, bad species or a general
        cell too small for the bead spread raise."""
        t0 = time.perf_counter()
        rounds = 0
        while True:
            st = self.nl.status(clear=True)
            flags, mr, ma = st["flags"], st["max_union_radial"], st["max_union_angular"]
            wf = self.ws.poll(clear=True)
            st3 = self.d3_nl.status(clear=True) if self.d3_nl is not None else None
            if st3 is not None:
                flags |= st3["flags"] & ~lib.FLAG_NEIGHBOR_OVERFLOW
            over = bool(st["flags"] & lib.FLAG_NEIGHBOR_OVERFLOW)
            over3 = st3 is not None and bool(st3["flags"] & lib.FLAG_NEIGHBOR_OVERFLOW)
            if not (over or over3):
                self.rebuilds_total += int(st["rebuilds"])
                break
            spent = time.perf_counter() - t0
            if rounds >= self.max_regrow or spent > self.regrow_budget_s:
                raise lib.NepError(5, f"candidate rows still overflow at step {self.step_no} after {rounds} "
                                      f"regrowths in {spent:.1f} s: capacities {self.caps} (D3 {self.d3_caps}), "
                                      f"longest rows ({st['max_cand_radial']}, {st['max_cand_angular']}), "
                                      f"snapshot at step {self._snap['step_no']}")
            self._grow_and_replay(st if over else None, st3 if over3 else None)
            rounds += 1
        if (flags | wf) & lib.FLAG_NONFINITE:
            raise lib.NepError(6, "non-finite force or position")
        if (flags | wf) & lib.FLAG_BAD_TYPE:
            raise lib.NepError(1, "species index outside the model's range")
        if flags & lib.FLAG_CELL_TOO_SMALL:
            raise lib.NepError(4, "general cell: the smallest face distance is below the candidate radius "
                                  "rc + 2 D + skin")
        self._snapshot()
        return mr, ma

    def _snapshot(self):
        """Device copy of the state at a verified point (positions, velocities,
        cell, step, recorded observables)."""
        self._snap = dict(step_no=self.step_no, started=self.started, pos=self.pos.clone(), vel=self.vel.clone(),
                          box=np.array(self.box, dtype=np.float64, copy=True), obs_n=len(self.obs_log),
                          dump_n=len(self.dump_log), rdf_frames=self.rdf_frames,
                          rdf=None if self.rdf_hist is None else self.rdf_hist.clone(),
                          extra=[save() for save, _ in self.snapshot_hooks])

    @staticmethod
    def _grown(caps, st):
        # rows found after an overflow may come from a state that truncated forces
        # spoiled: grow by at most 2x (a replay that still overflows grows again)
        need = (int(np.ceil(st["max_cand_radial"] * 1.25)) + 8, int(np.ceil(st["max_cand_angular"] * 1.25)) + 8)
        return tuple(max(a + 1, min(b, 2 * a)) for a, b in zip(caps, need))

    def _grow_and_replay(self, st, st3=None):
        if st is not None:
            self.caps = self._grown(self.caps, st)
            self.nl = lib.NeighborList(self.model, self.P, self.N, *self.caps,
                                       offsets=self.offsets if self.batched else None)
            self.nl.set_skin(self.skin)
        if st3 is not None:
            self.d3_caps = self._grown(self.d3_caps, st3)
            self.d3_nl = lib.NeighborList(self.d3.list_model, self.P, self.N, *self.d3_caps)
            self.d3_nl.set_skin(self.skin)
        had_graph = self.graph is not None
        self.graph = None
        target = self.step_no
        s = self._snap
        self.pos.copy_(s["pos"])
        self.vel.copy_(s["vel"])
        self.box = s["box"].copy()
        self.step_no, self.started = s["step_no"], s["started"]
        del self.obs_log[s["obs_n"]:]
        del self.dump_log[s["dump_n"]:]
        self.rdf_frames = s["rdf_frames"]
        if self.rdf_hist is not None:
            self.rdf_hist.copy_(s["rdf"])
        for (_, restore), tok in zip(self.snapshot_hooks, s["extra"]):
            restore(tok)
        self.rollbacks += 1
        # replay the same calls: steps, then finish() or a fresh capture (whose
        # own eager step is the last one) where the original sequence had them
        finished = self._finished
        last = target - 1 if (finished or had_graph) else target
        every, self.check_every = self.check_every, 0   # the caller's poll verifies the replay
        one = self.replay_step or self.step
        try:
            while self.step_no < last:
                one()
            if finished:
                self.finish()
            elif had_graph:
                self.capture(self.graph_steps)
        finally:
            self.check_every = every

    def start(self):
        self.forces()
        self.pimd.step(self.pos, self.vel, self.F, self.step_no, lib.PRE)
        self.started = True

    def _split(self) -> bool:
        return bool(self.obs_every or self.baro or self.dump_every)

    def _after_forces(self, n: int):
        """Partial RDF counts from the lists of step n's force call."""
        c = self.rdf_cfg
        if c and (n + 1) % int(c.get("every", 1)) == 0:
            self.nl.rdf_accumulate(self.pos, self.box, self.types, self.rdf_hist, c["rmax"])
            self.rdf_frames += 1

    def _after_post(self, n: int):
        """Observables, velocity dump and pressure control between the closing half of step n and the next step."""
        if self.dump_every and (n + 1) % self.dump_every == 0:
            out = self.torch.empty((self.N, 3), dtype=self.torch.float64, device=self.pos.device)
            self.pimd.centroid(self.vel, out)
            self.dump_log.append((n, out))
        rec = self.obs_every and (n + 1) % self.obs_every == 0
        if not (rec or self.baro):
            return
        self.pimd.observables(self.pos, self.F, self.W, self.E, self.box, self.obs)
        if rec:
            self.obs_log.append((n, self.obs.clone()))
        if self.baro:
            b = self.baro
            self.pimd.berendsen(self.pos, self.obs, self.mu, p0=b["p0"], beta=b["beta"], tau_p=b["tau_p"],
                                anisotropic=b.get("anisotropic", False))
            mu = self.mu.cpu().numpy()     # the next neighbour build needs the new cell
            if not (np.all(np.isfinite(mu)) and np.all(mu > 0.0)):
                raise lib.NepError(6, f"barostat scaling factors {mu}")
            # every Cartesian component a of the positions and of the edge vectors scales by mu_a
            box = np.asarray(self.box, np.float64)
            self.box = box * mu if box.shape == (3,) else (box.reshape(3, 3) * mu[None, :]).reshape(box.shape)

    def step(self):
        """One full step, launched eagerly: forces at the advanced positions,
        then POST(n) + PRE(n+1).  (`run` replays a captured graph where it can.)"""
        self._finished = False
        if not self.started:
            self.start()
        fold = self._fold()
        self.forces(defer=fold)
        n = self.step_no
        if self.on_forces is not None:
            self.on_forces(n)
        self._after_forces(n)
        if self._split():
            self.pimd.step(self.pos, self.vel, self.F, n, lib.POST)
            self._after_post(n)
            self.pimd.step(self.pos, self.vel, self.F, n + 1, lib.PRE)
        elif fold:   # the E/W sums ride in the integrator launch
            self.pimd.step_nep(self.pos, self.vel, self.F, n, lib.FUSED, self.ws)
        else:
            self.pimd.step(self.pos, self.vel, self.F, n, lib.FUSED)
        self.step_no += 1
        if self.graph is not None:
            self._dev_stale = True
        if self.check_every and self.step_no % self.check_every == 0:
            self.check()

    def run(self, n: int):
        """n steps: replays of the captured graph while at least its step count
        remains, eager steps otherwise."""
        while n > 0:
            if self.graph is not None and n >= self.graph_steps:
                self._finished = False
                if self._dev_stale:
                    self.step_dev[0].fill_(self.step_no)   # the counter the graph reads first
                    self._dev_stale = False
                before = self.step_no
                self.graph.replay()
                self.step_no += self.graph_steps
                n -= self.graph_steps
                if self.check_every and self.step_no // self.check_every != before // self.check_every:
                    self.check()
            else:
                self.step()
                n -= 1

    def capture(self, steps: int = 2):
        """Capture `steps` full steps (lists, forces, fused integrator stage;
        an even number) as one HIP graph, replayed by `run`.

        The step number lives in two device counters that the captured
        integrator launches read and write alternately, so every replay draws
        fresh noise with no extra launch; one replay's launch overhead is
        shared by its steps.  The box and the species must stay fixed while
        the graph is in use; `release()` returns to eager launches."""
        t = self.torch
        if steps < 2 or steps % 2:
            raise ValueError("capture: the number of captured steps must be even (the step counters alternate)")
        if self._split() or self.rdf_cfg:
            raise ValueError("capture: observables, dumps, RDFs and the barostat run eagerly")
        self.graph = None
        if not self.started:
            self.start()
        # one eager step first so that every lazy allocation has happened
        self.step()
        self.step_dev = t.tensor([self.step_no, 0], dtype=t.int64, device=self.pos.device)
        c = (self.step_dev[0:1], self.step_dev[1:2])
        t.cuda.synchronize()
        g = t.cuda.CUDAGraph()
        fold = self._fold()
        with t.cuda.graph(g):
            for k in range(steps):
                self.forces(defer=fold)
                if fold:
                    self.pimd.step_nep(self.pos, self.vel, self.F, 0, lib.FUSED, self.ws, c[k % 2], c[(k + 1) % 2])
                else:
                    self.pimd.step_dev(self.pos, self.vel, self.F, c[k % 2], c[(k + 1) % 2], lib.FUSED)
        t.cuda.synchronize()
        # capture does not execute: the counters and the state are unchanged
        self.graph = g
        self.graph_steps = steps
        self._dev_stale = False

    def release(self):
        self.graph = None

    def finish(self):
        """Close the current step (forces + POST), leaving synchronised q and v."""
        self.graph = None
        if not self.started:
            self.start()
        self.forces()
        self._after_forces(self.step_no)
        self.pimd.step(self.pos, self.vel, self.F, self.step_no, lib.POST)
        self._after_post(self.step_no)
        self.started = False
        self.step_no += 1
        self._finished = True

    def rdf(self):
        """Partial radial distribution functions from the accumulated counts
        (synchronises): bin centres [nbins] and g [S, S, nbins], normalised by
        frames x P x N_a x (N_b - [a == b]) / V x shell volume, V the current
        cell volume.  Also returns the raw counts."""
        if not self.rdf_cfg:
            raise ValueError("the engine was created without rdf=")
        counts = self.rdf_hist.cpu().numpy().astype(np.uint64)
        types = self.types.cpu().numpy()
        n_sp = [int((types == a).sum()) for a in range(self.model.n_species)]
        vol = I.cell_volume(self.box)
        r, g = rdf_normalise(counts, n_sp, vol, float(self.rdf_cfg["rmax"]), self.rdf_frames, self.P)
        return r, g, counts

    def centroid_velocities(self):
        """Dumped centroid velocities (synchronises): steps [n] and [n, N, 3] (A/fs)."""
        if not self.dump_log:
            return np.zeros(0, np.int64), np.zeros((0, self.N, 3))
        steps = np.array([n for n, _ in self.dump_log], np.int64)
        return steps, self.torch.stack([v for _, v in self.dump_log]).cpu().numpy()

    def observables_history(self):
        """Recorded observables (synchronises): steps [n] and the vectors [n, OBS_COUNT]."""
        if not self.obs_log:
            return np.zeros(0, np.int64), np.zeros((0, lib.OBS_COUNT))
        steps = np.array([n for n, _ in self.obs_log], np.int64)
        return steps, self.torch.stack([o for _, o in self.obs_log]).cpu().numpy()
