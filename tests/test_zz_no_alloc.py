"""The allocation-free fused step (rb_rigid_step_fused_noalloc) against the
workspace form (rb_rigid_step_fused), through the C ABI: the same state in,
the same bits out, on two calls in a row -- the second on a smaller system,
so that the shared scratch array holds the first call's partial sums -- and
the size limit reported as an error."""
import ctypes

import numpy as np
import pytest

from synth import configs, state

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def abi():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_12199_amd import abi as _abi
    return _abi


def _state_with_forces(abi, cfg, n_keep):
    """A system of the first n_keep bodies of the workload, its bead forces
    added into the accumulator (the input of a fused step boundary)."""
    from paper_2402_12199_amd.md import RigidSystem
    st = state.initial_state(cfg)
    b = cfg.body
    sysm = RigidSystem([b.beads], [b.mass], [b.inertia], st["types"][:n_keep], st["x"][:n_keep], st["q"][:n_keep],
                       st["P"][:n_keep], st["L"][:n_keep], cfg.box, cfg.r_list, cfg.skin)
    sysm.init_forces("bead")          # list, forces, finalize (accumulator cleared)
    sysm.bead_forces()                # this step's forces into the accumulator
    torch.cuda.synchronize()
    return sysm


FIELDS = ("x", "P", "q", "L", "acc", "force", "torque", "ev", "kinetic", "flags", "x_ref")


def _copy(sysm):
    return {k: getattr(sysm, k).clone() for k in FIELDS}


def _step(abi, sysm, buf, dt, noalloc, ws=None):
    args = (sysm.ctx, dt, buf["x"], buf["P"], buf["q"], buf["L"], sysm.types, buf["acc"], buf["force"], buf["torque"],
            buf["ev"], buf["x_ref"], sysm.half_skin, buf["kinetic"], buf["flags"])
    if noalloc:
        abi.rb_rigid_step_fused_noalloc(*args)
    else:
        abi.rb_rigid_step_fused(*args, ws)


def test_noalloc_fused_step_matches_workspace_form_on_two_calls(abi):
    cfg = configs.config1()
    dt = cfg.dt
    for n_keep in (64, 40):            # second call: a smaller input
        sysm = _state_with_forces(abi, cfg, n_keep)
        ref, got = _copy(sysm), _copy(sysm)
        ws = torch.zeros(abi.rb_rigid_workspace_bytes(sysm.n), dtype=torch.uint8, device="cuda")
        _step(abi, sysm, ref, dt, noalloc=False, ws=ws)
        _step(abi, sysm, got, dt, noalloc=True)
        torch.cuda.synchronize()
        for k in FIELDS:
            assert torch.equal(ref[k], got[k]), (n_keep, k)
        # the step did something: the kinetic energy was reduced and the
        # accumulator converted and cleared
        assert float(got["kinetic"].sum()) > 0.0
        assert int(torch.count_nonzero(got["acc"])) == 0
        assert not torch.equal(got["x"], sysm.x)


def test_noalloc_fused_step_rejects_sizes_beyond_its_scratch(abi):
    from paper_2402_12199_amd import _lib
    cfg = configs.config1()
    b = cfg.body
    ctx = abi.Ctx([b.beads], [b.mass], [b.inertia])
    lim = abi.rb_rigid_step_fused_noalloc_max_bodies()
    assert lim == 1 << 22
    # rejected before any device access: stand-in addresses are never used
    fake = ctypes.c_void_p(4096)
    L = _lib.lib()
    rc = L.rb_rigid_step_fused_noalloc(ctx.handle, lim + 1, 0.005, fake, fake, fake, fake, fake, fake, fake, fake,
                                       None, None, 0.5, None, None, 0.0, None, fake, None)
    assert rc == abi.RB_ERR_INVALID_ARG
    assert "scratch limit" in L.rb_last_error().decode()
