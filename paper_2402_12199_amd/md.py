"""Dynamics driver: composes the C-ABI entry points into one MD step.

Bead path step (velocity Verlet):
  rigid_step phase 1 (half kick, drift, free rotation, skin and margin tests)
  pairlist_build (only when the skin test flagged a rebuild)
  bead_pair_forces over every listed pair (optionally after bead_screen), or
  bead_pair_forces_screened (two-level list: the listed pairs whose bead
  boxes came within rc + margin at the last screening)
  -> accum_finalize (which also clears the accumulator for the next step)
  rigid_step phase 2 (second half kick, kinetic energy)
Network path step: the same, except that after the pair list
  pair_descriptors routes each pair to the network (|d| >= d_min) or to the
  bead sum, and nn_pair_forces + bead_pair_forces share one accumulator.

Every call only enqueues work on the current stream; nothing in `step`
synchronises, so a step can be captured in a HIP graph.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import abi


@dataclass
class NNModel:
    params: torch.Tensor           # RB_MLP_NPARAMS FP32 on the device
    norm: np.ndarray               # 16 floats
    precision: int = abi.RB_PREC_BF16
    d_min: float = 0.0             # below: bead fallback
    sw_lo: float = 0.0             # energy switch (sw_hi <= sw_lo: off)
    sw_hi: float = 0.0
    sym: bool = False              # network takes the symmetry-reduced cube-pair descriptor
    form: str = "dq"               # network input: "dq" (d, q), "cube" (= sym) or "cyl" (four-number form)
    gap_min: float | None = None   # shells' bound on the closest bead distance below which the bead sum takes over
    gap_max: float | None = None   # bound at or above which a pair is skipped (no bead pair within it)

    def __post_init__(self):
        if self.sym:
            self.form = "cube"
        self.sym = self.form == "cube"
        if self.form not in ("dq", "cube", "cyl"):
            raise ValueError(f"unknown network input form {self.form}")


class RigidSystem:
    def __init__(self, templates, masses, inertias, types, x, q, P, L, box, r_list, skin,
                 eps=1.0, sigma=1.0, rc=2.5, max_pairs=None, device="cuda", screen=False, hphc=None,
                 margin=None, nvt=None):
        """hphc: dict(A, b, c, p) selects the half-power half-cosine bead
        potential instead of Lennard-Jones (r_list must then cover its
        cutoff b + pi / c).  margin: two-level lists rebuilt when a body's
        beads may have moved by margin / 2 -- the bead path's screened pairs
        (rb_bead_pair_forces_screened) or the network path's routing
        candidates (rb_pair_descriptors_screened); both use the rescreen
        flag, so a system takes one of the two.  nvt: dict(kT, tau) runs
        the plain steps at constant temperature (Nose-Hoover, g = 6 n - 3,
        Q = g kT tau^2)."""
        if screen and margin is not None:
            raise ValueError("screen and margin are exclusive")
        self.dev = torch.device(device)
        self.ctx = abi.Ctx(templates, masses, inertias, eps, sigma, rc)
        if hphc is not None:
            self.ctx.set_hphc(**hphc)
        n = len(x)
        self.n = n
        self.box = np.broadcast_to(np.asarray(box, np.float64), (3,)).copy()
        self.r_list = float(r_list)
        self.half_skin = 0.5 * float(skin)

        def dt64(a, rows):
            return torch.tensor(np.ascontiguousarray(np.asarray(a, np.float64).T.reshape(rows, n)),
                                device=self.dev)

        self.x = dt64(x, 3)
        self.q = dt64(q, 4)
        self.P = dt64(P, 3)
        self.L = dt64(L, 3)
        self.types = torch.tensor(np.asarray(types, np.int32), device=self.dev)
        self.x_ref = torch.zeros_like(self.x)
        self.flags = torch.zeros(abi.RB_NFLAGS, dtype=torch.int32, device=self.dev)
        if max_pairs is None:
            vol = float(np.prod(self.box))
            mean_nb = n * 4.0 / 3.0 * math.pi * self.r_list ** 3 / vol
            max_pairs = int(n * (4.0 * mean_nb + 8.0) / 2.0) + 4096
        self.max_pairs = int(max_pairs)
        self.pair_i = torch.zeros(self.max_pairs, dtype=torch.int32, device=self.dev)
        self.pair_j = torch.zeros(self.max_pairs, dtype=torch.int32, device=self.dev)
        self.acc = torch.zeros(abi.acc_len(n), dtype=torch.int64, device=self.dev)
        abi.rb_accum_zero(n, self.acc)
        self.force = torch.zeros((3, n), dtype=torch.float32, device=self.dev)
        self.torque = torch.zeros((3, n), dtype=torch.float32, device=self.dev)
        self.ev = torch.zeros(10, dtype=torch.float64, device=self.dev)
        self.kinetic = torch.zeros(2, dtype=torch.float64, device=self.dev)
        self.ws_pl = torch.zeros(abi.rb_pairlist_workspace_bytes(n, self.box, self.r_list), dtype=torch.uint8,
                                 device=self.dev)
        self.ws_rig = torch.zeros(abi.rb_rigid_workspace_bytes(n), dtype=torch.uint8, device=self.dev)
        self.nn: NNModel | None = None
        self.desc = None
        # optional bead-path screen (a separate pass over the list that keeps
        # the pairs whose bead boxes can interact; the force kernel applies
        # the same test itself, so the screen pays off only when most listed
        # pairs are far apart)
        self.screen = screen
        self.idx_screen = torch.zeros(self.max_pairs, dtype=torch.int32, device=self.dev)
        self.tmp_screen = torch.zeros(2, dtype=torch.int32, device=self.dev)
        # two-level list
        self.margin = None if margin is None else float(margin)
        self.x_sref = self.q_sref = None
        if self.margin is not None:
            self.screen_list = torch.zeros(self.max_pairs, dtype=torch.int32, device=self.dev)
            self.cand_list = torch.zeros(self.max_pairs, dtype=torch.int32, device=self.dev)
            self._two_level = None   # "bead" or "route": the user of the rescreen flag
            self.x_sref = torch.zeros_like(self.x)
            self.q_sref = torch.zeros_like(self.q)
            self.tmp_two = torch.zeros(4, dtype=torch.int32, device=self.dev)
            self.flags[abi.RB_FLAG_RESCREEN] = 1
        self.half_margin = 0.0 if margin is None else 0.5 * float(margin)
        # Nose-Hoover state (xi, eta, s, Q, g kT)
        self.nh = None
        if nvt is not None:
            g = 6.0 * n - 3.0
            kT, tau = float(nvt["kT"]), float(nvt["tau"])
            self.nh = torch.tensor([0.0, 0.0, 1.0, g * kT * tau * tau, g * kT], dtype=torch.float64, device=self.dev)

    # ------------------------------------------------------------ pieces
    def build_pairs(self, always=True):
        abi.rb_pairlist_build(self.x, self.box, self.r_list, self.pair_i, self.pair_j, self.x_ref, self.flags,
                              abi.RB_BUILD_ALWAYS if always else abi.RB_BUILD_IF_FLAGGED, self.ws_pl)

    def set_nn(self, model: NNModel):
        self.nn = model
        self.desc = torch.zeros((7, self.max_pairs), dtype=torch.float32, device=self.dev)
        self.idx_nn = torch.zeros(self.max_pairs, dtype=torch.int32, device=self.dev)
        self.idx_bead = torch.zeros(self.max_pairs, dtype=torch.int32, device=self.dev)
        if model.sym:
            self.sym = torch.zeros((7, self.max_pairs), dtype=torch.float32, device=self.dev)
            self.jac = torch.zeros((49, self.max_pairs), dtype=torch.float32, device=self.dev)

    def _take_two_level(self, user):
        if self._two_level is None:
            self._two_level = user
        elif self._two_level != user:
            raise RuntimeError(f"this system's two-level list serves the {self._two_level} path; "
                               f"the {user} path needs a system of its own")

    def route(self, d_min, d_max, gap_min=None, gap_max=None, two_level=True):
        """Descriptors of the listed pairs and their routing (network, bead
        sum, neither); with gap_min the shells' bound on the closest bead
        distance routes as well, and with a margin (two-level list) only the
        candidates of the last screening are routed (two_level=False: every
        listed pair)."""
        shells = gap_min is not None
        if two_level and shells and self.margin is not None and gap_max is not None and gap_max > 0:
            # two-level routing: the candidates of the last screening only
            self._take_two_level("route")
            abi.rb_pair_descriptors_screened(self.x, self.q, self.box, self.pair_i, self.pair_j, d_min, self.desc,
                                             self.idx_nn, self.idx_bead, self.flags, d_max, self.ctx, self.types,
                                             gap_min, gap_max, self.margin, self.cand_list, self.x_sref,
                                             self.q_sref)
            return
        abi.rb_pair_descriptors(self.x, self.q, self.box, self.pair_i, self.pair_j, d_min, self.desc, self.idx_nn,
                                self.idx_bead, self.flags, d_max=d_max, ctx=self.ctx if shells else None,
                                types=self.types if shells else None, gap_min=gap_min if shells else 0.0,
                                gap_max=gap_max if shells and gap_max is not None else 0.0)

    def nn_forces(self):
        """Descriptors, routing, network forces of the routed pairs and the
        bead sum of the fallback pairs, all into the accumulator."""
        m = self.nn
        self.route(m.d_min, m.sw_hi if m.sw_hi > m.sw_lo else 0.0, m.gap_min, m.gap_max)
        if m.form in ("cyl", "dq"):
            # network pairs and bead-sum pairs in one call (one launch in BF16)
            abi.rb_nn_pair_forces_routed(self.ctx, m.params, m.norm, m.precision, 1 if m.form == "cyl" else 0, self.x,
                                         self.q, self.types, self.box, self.pair_i, self.pair_j, self.desc,
                                         self.idx_nn, self.flags[abi.RB_FLAG_NNN:], self.idx_bead,
                                         self.flags[abi.RB_FLAG_NBEAD:], self.max_pairs, m.sw_lo, m.sw_hi, self.acc,
                                         self.flags)
            return
        if m.form == "cube":
            abi.rb_cube_sym_descriptors(self.desc, self.sym, self.jac, self.idx_nn, self.flags[abi.RB_FLAG_NNN:],
                                        self.max_pairs)
            abi.rb_nn_pair_forces_sym(m.params, m.norm, m.precision, self.q, self.pair_i, self.pair_j, self.desc,
                                      self.sym, self.jac, self.idx_nn, self.flags[abi.RB_FLAG_NNN:], self.max_pairs,
                                      m.sw_lo, m.sw_hi, self.acc, self.flags)
        abi.rb_bead_pair_forces(self.ctx, self.x, self.q, self.types, self.box, self.pair_i, self.pair_j,
                                self.idx_bead, self.flags[abi.RB_FLAG_NBEAD:], self.max_pairs, self.acc, self.flags)

    def bead_forces(self):
        """Bead sum over the whole list (or over the screened pairs)."""
        if self.margin is not None:
            self._take_two_level("bead")
            abi.rb_bead_pair_forces_screened(self.ctx, self.x, self.q, self.types, self.box, self.pair_i,
                                             self.pair_j, self.flags[abi.RB_FLAG_NPAIRS:], self.max_pairs,
                                             self.margin, self.screen_list, self.x_sref, self.q_sref, self.tmp_two,
                                             self.acc, self.flags)
            return
        if not self.screen:
            abi.rb_bead_pair_forces(self.ctx, self.x, self.q, self.types, self.box, self.pair_i, self.pair_j,
                                    None, self.flags[abi.RB_FLAG_NPAIRS:], self.max_pairs, self.acc, self.flags)
            return
        abi.rb_bead_screen(self.ctx, self.x, self.q, self.types, self.box, self.pair_i, self.pair_j, None,
                           self.flags[abi.RB_FLAG_NPAIRS:], self.max_pairs, self.idx_screen,
                           self.flags[abi.RB_FLAG_NSCREEN:], self.tmp_screen, self.flags)
        abi.rb_bead_pair_forces(self.ctx, self.x, self.q, self.types, self.box, self.pair_i, self.pair_j,
                                self.idx_screen, self.flags[abi.RB_FLAG_NSCREEN:], self.max_pairs, self.acc,
                                self.flags)

    def compute_forces(self, path="bead"):
        # the accumulator is clear: zeroed at construction, cleared again by
        # every rb_accum_finalize
        if path == "bead":
            self.bead_forces()
        elif path == "nn":
            self.nn_forces()
        else:
            raise ValueError(path)
        abi.rb_accum_finalize(self.n, self.acc, self.force, self.torque, self.ev, self.flags)

    def init_forces(self, path="bead"):
        self.build_pairs(always=True)
        self.compute_forces(path)

    def step(self, dt, path="bead"):
        abi.rb_rigid_step(self.ctx, 1, dt, self.x, self.P, self.q, self.L, self.types, self.force, self.torque,
                          self.x_ref, self.half_skin, None, self.flags, None, self.x_sref, self.q_sref,
                          self.half_margin, nh=self.nh)
        self.build_pairs(always=False)
        self.compute_forces(path)
        abi.rb_rigid_step(self.ctx, 2, dt, None, self.P, self.q, self.L, self.types, self.force, self.torque,
                          None, 0.0, self.kinetic, None, self.ws_rig, nh=self.nh)

    def extended_energy(self) -> float:
        """After a step: K + U + Q xi^2 / 2 + g kT eta with K the kinetic
        energy of the thermostat-scaled momenta (conserved by the
        thermostatted dynamics); K + U without a thermostat."""
        K = float(self.kinetic.sum().item())
        if self.nh is None:
            return self.energy() + K
        xi, eta, s, Q, gkT = self.nh.cpu().numpy()
        return self.energy() + s * s * K + 0.5 * Q * xi * xi + gkT * eta

    # ------------------------------------------------------------ fused loop
    def _forces_to_acc(self, path):
        if path == "bead":
            self.bead_forces()
        else:
            self.nn_forces()

    def begin_fused(self, dt):
        """Phase 1 of the first step of a fused run (forces must be current)."""
        if self.nh is not None:
            raise ValueError("the fused step is constant-energy only; thermostatted runs use step()")
        abi.rb_rigid_step(self.ctx, 1, dt, self.x, self.P, self.q, self.L, self.types, self.force, self.torque,
                          self.x_ref, self.half_skin, None, self.flags, None, self.x_sref, self.q_sref,
                          self.half_margin)

    def fused_step(self, dt, path="bead", kinetic=False):
        """Pair list, forces into the accumulator, then one launch for the end
        of this step and the start of the next (see rb_rigid_step_fused).
        The kinetic energy is reduced only when asked for (end_fused always
        does)."""
        if self.nh is not None:
            raise ValueError("the fused step is constant-energy only; thermostatted runs use step()")
        self.build_pairs(always=False)
        self._forces_to_acc(path)
        abi.rb_rigid_step_fused(self.ctx, dt, self.x, self.P, self.q, self.L, self.types, self.acc, self.force,
                                self.torque, self.ev, self.x_ref, self.half_skin,
                                self.kinetic if kinetic else None, self.flags, self.ws_rig, self.x_sref, self.q_sref,
                                self.half_margin)

    def end_fused(self, dt, path="bead"):
        """Last step of a fused run: forces, finalize, phase 2."""
        self.build_pairs(always=False)
        self.compute_forces(path)
        abi.rb_rigid_step(self.ctx, 2, dt, None, self.P, self.q, self.L, self.types, self.force, self.torque,
                          None, 0.0, self.kinetic, None, self.ws_rig)

    # ------------------------------------------------------------ graphs
    def capture(self, dt, path="bead", steps=1, fused=False, kinetic_last=True):
        """Record `steps` MD steps into a HIP graph (torch.cuda.CUDAGraph).

        Every step only enqueues kernels whose sizes are fixed at capture and
        whose data-dependent extents (pair counts, rebuild flag) are read on
        the device, so replaying the graph performs the same work as calling
        `step` that many times.  Capturing does not execute the steps.  With
        fused steps the kinetic energy is reduced in the graph's last step
        (kinetic_last), so a replay leaves the energy of its end state.
        """
        # one eager call first so lazily cached host values exist before capture
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            for k in range(steps):
                if fused:
                    self.fused_step(dt, path, kinetic=kinetic_last and k == steps - 1)
                else:
                    self.step(dt, path)
        torch.cuda.current_stream().wait_stream(side)
        return g

    def pair_configurations(self, d_min: float, d_max: float, gap_min=None, gap_max=None) -> torch.Tensor:
        """Descriptors (7, m) of the listed pairs the router sends to the
        network: d_min <= |d| < d_max and, with gap_min, a shells' bound on
        the closest bead distance in [gap_min, gap_max) (training data drawn
        from the dynamics; uses the routing buffers)."""
        if self.desc is None:
            self.desc = torch.zeros((7, self.max_pairs), dtype=torch.float32, device=self.dev)
            self.idx_nn = torch.zeros(self.max_pairs, dtype=torch.int32, device=self.dev)
            self.idx_bead = torch.zeros(self.max_pairs, dtype=torch.int32, device=self.dev)
        self.route(d_min, d_max, gap_min, gap_max, two_level=False)
        m = int(self.flags[abi.RB_FLAG_NNN].item())
        idx = torch.sort(self.idx_nn[:m].long()).values   # list order, independent of append order
        return self.desc[:, idx]

    # ------------------------------------------------------------ readback
    def flags_host(self) -> np.ndarray:
        return self.flags.cpu().numpy()

    def check_capacity(self):
        """Raises on any condition the device reported (pair-list overflow,
        non-finite forces, fixed-point overflow, quaternion drift), through
        rb_flags_check; returns the host copy of the flags."""
        f = self.flags_host()
        rc, msg = abi.rb_flags_check(f)
        if rc != abi.RB_OK:
            raise RuntimeError(f"{msg} (capacity {self.max_pairs})" if rc == abi.RB_ERR_CAPACITY else msg)
        return f

    def state_host(self) -> dict:
        return dict(x=self.x.cpu().numpy().T.copy(), q=self.q.cpu().numpy().T.copy(),
                    P=self.P.cpu().numpy().T.copy(), L=self.L.cpu().numpy().T.copy())

    def energy(self) -> float:
        return float(self.ev[0].item())

    def kinetic_host(self) -> np.ndarray:
        return self.kinetic.cpu().numpy()

    def pairs_host(self) -> np.ndarray:
        npairs = int(self.flags[abi.RB_FLAG_NPAIRS].item())
        return np.stack([self.pair_i[:npairs].cpu().numpy(), self.pair_j[:npairs].cpu().numpy()], axis=1)
