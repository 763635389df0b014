"""Pins of the constant-temperature oracle (Nose-Hoover thermostat around
the rigid-body integrator; the paper states only that its runs are
Nose-Hoover NVT, section 3) against the constant-energy integrator, the
continuous thermostat equations solved independently, and the conserved
quantity."""
import numpy as np
from scipy.integrate import solve_ivp

from oracle import beads, thermostat
from synth import configs, state


def _copy(st):
    return {k: np.ascontiguousarray(st[k].copy()) for k in ("x", "P", "q", "L")}


def test_infinite_thermostat_mass_is_the_constant_energy_integrator():
    cfg = configs.config1()
    st = state.initial_state(cfg)
    b = cfg.body
    a, c = _copy(st), _copy(st)
    steps = 15
    r = beads.nve(a["x"], a["P"], a["q"], a["L"], st["types"], [b.beads], [b.mass], [b.inertia], cfg.box, steps,
                  cfg.dt)
    g = 6.0 * cfg.n_bodies - 3.0
    o = thermostat.nvt(c["x"], c["P"], c["q"], c["L"], st["types"], [b.beads], [b.mass], [b.inertia], cfg.box, steps,
                       cfg.dt, Q=1e300, gkT=g * 1.5)
    assert np.all(o["scale"] == 1.0)
    for k in ("x", "P", "q", "L"):
        assert np.array_equal(a[k], c[k]), k
    assert np.array_equal(o["ke"], r["ke"][1:])


def _free_run(dt, t_end, kT, tau):
    # 27 isotropic cube bodies far apart (no bead pair within rc): the
    # velocity-Verlet part keeps K fixed and the run is the thermostat alone
    body = configs.cube5()
    n = 27
    grid = np.stack(np.meshgrid(*[np.arange(3)] * 3, indexing="ij"), -1).reshape(-1, 3) * 100.0
    rng = np.random.default_rng(3)
    x = np.ascontiguousarray(grid.astype(np.float64))
    P = rng.normal(size=(n, 3)) * np.sqrt(body.mass)
    P -= P.mean(axis=0)
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    L = rng.normal(size=(n, 3)) * np.sqrt(body.inertia)
    g = 6.0 * n - 3.0
    Q = g * kT * tau * tau
    steps = int(round(t_end / dt))
    o = thermostat.nvt(x, P, q, L, np.zeros(n, np.int32), [body.beads], [body.mass], [body.inertia], None, steps,
                       dt, Q=Q, gkT=g * kT)
    return o, Q, g


def test_free_bodies_follow_the_thermostat_equations():
    kT, tau, t_end = 2.0, 0.3, 1.5
    assert np.allclose(configs.cube5().inertia, configs.cube5().inertia[0])   # isotropic: free rotation keeps K
    errs = []
    for dt in (0.01, 0.005):
        o, Q, g = _free_run(dt, t_end, kT, tau)
        assert np.all(o["pe"] == 0.0)
        K0 = o["ke"][0]
        # dK/dt = -2 xi K, dxi/dt = (2K - g kT) / Q from K0, xi = 0
        sol = solve_ivp(lambda t, y: [-2.0 * y[1] * y[0], (2.0 * y[0] - g * kT) / Q], (0.0, t_end), [K0, 0.0],
                        rtol=1e-12, atol=1e-12)
        K_ref, xi_ref = sol.y[0, -1], sol.y[1, -1]
        K_end = o["ke"][-1] * o["scale"][-1] ** 2
        errs.append(max(abs(K_end - K_ref) / K_ref, abs(o["xi"][-1] - xi_ref) / max(abs(xi_ref), 1e-12)))
    assert errs[1] < 1e-3
    assert 3.0 < errs[0] / errs[1] < 5.0          # second order in dt


def test_hot_start_cools_toward_the_target():
    o, Q, g = _free_run(0.005, 1.0, kT=0.5, tau=0.3)
    T = 2.0 * o["ke"] / g
    assert T[0] > 0.9 and T[-1] < T[0]             # started near kT = 1, pulled toward 0.5
    assert o["xi"][:20].min() > 0                  # friction switches on while too hot


def _conserved_dev(cfg, st, dt, t_end):
    b = cfg.body
    c = _copy(st)
    g = 6.0 * cfg.n_bodies - 3.0
    steps = int(round(t_end / dt))
    o = thermostat.nvt(c["x"], c["P"], c["q"], c["L"], st["types"], [b.beads], [b.mass], [b.inertia], cfg.box,
                       steps, dt, Q=g * 1.5 * 0.2 ** 2, gkT=g * 1.5)
    assert abs(o["xi"]).max() > 0.1                # the thermostat does real work
    assert np.count_nonzero(o["pe"]) > 0
    return np.abs(o["conserved"] - o["conserved"][0]).max() / o["ke"].mean()


def test_conserved_quantity_with_interactions():
    cfg = configs.config1()
    st = state.initial_state(cfg)
    # Lennard-Jones shifted in energy only: the force jumps at rc, so bead
    # pairs crossing it add errors of order dt; the bound still holds
    assert _conserved_dev(cfg, st, 0.002, 0.8) < 1e-3
    # half-power half-cosine: force continuous at rc, the deviation falls
    # like dt^2
    with beads.use_hphc(**beads.HPHC_PAPER):
        devs = [_conserved_dev(cfg, st, dt, 0.8) for dt in (0.004, 0.002)]
    assert devs[1] < 1e-3
    assert 3.0 < devs[0] / devs[1] < 5.0
