"""Plant plausible mistakes in copies of the oracle and check that the pins
catch every one of them.

Each mutation replaces one snippet of the oracle source (it must occur
exactly once), the mutated source is executed as a fresh module, and the pins
are run against it; at least one must fail.
"""
import os
import sys
import types

import pytest

import pins
import test_oracle_pins as checks

ORACLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "oracle", "worm_lbm.py")

MUTATIONS = {
    "dded_moves_on_pause": (
        "                self._deposit(acc, dded, 0, 0)",
        "                self._deposit(acc, dded, sx, sy)"),
    "eed_stays_on_pause": (
        "            self._deposit(acc, eed, sx, sy)",
        "            self._deposit(acc, eed, *((sx, sy) if hp[i] else (0, 0)))"),
    "tas_radius_without_extra_cell": (
        "h = cx * cx + cy * cy <= (n + 1) * (n + 1)",
        "h = cx * cx + cy * cy <= n * n"),
    "tas_tests_position_before_move": (
        "            cx = P[i][0] + D2Q8[m][0]\n            cy = P[i][1] + D2Q8[m][1]",
        "            cx = P[i][0]\n            cy = P[i][1]"),
    "worm_index_advances_on_pause": (
        "                P[i] = [cx, cy]\n                k[i] += 1",
        "                P[i] = [cx, cy]\n            k[i] += 1"),
    "equilibrium_ignores_weights": (
        "eed = Wc * self.w[i] * E",
        "eed = Wc * E / c.q"),
    "no_scattering_between_directions": (
        "eed = Wc * self.w[i] * E",
        "eed = Wc * self.e[i]"),
    "dded_not_relaxed": (
        "dded = (1.0 - Wc) * self.e[i]",
        "dded = self.e[i]"),
    "diffuse_wall_not_normalised": (
        "Tg = r / C",
        "Tg = r"),
    "diffuse_emission_wrong_row": (
        "e[i, yrow, :] += acc[1:nx + 1]",
        "e[i, yrow + dy_in, :] += acc[1:nx + 1]"),
    "periodic_x_wraps_to_wrong_side": (
        "            a[:, nx] += a[:, 0]",
        "            a[:, 1] += a[:, 0]"),
    "one_sided_weight_gap": (
        "w[j] = (up + dn) / (4.0 * math.pi)",
        "w[j] = up / (2.0 * math.pi)"),
    "ring_speed_not_per_hop": (
        "return math.hypot(vx, vy) / self.ring_m",
        "return math.hypot(vx, vy)"),
    "w_corr_without_ballistic_part": (
        "Wc = f * ((1.0 - W) * W + W * (W * self.lam))",
        "Wc = f * (W * (W * self.lam))"),
    "heat_flux_components_swapped": (
        "qx = np.tensordot(self.s[:, 0], self.e, axes=(0, 0))",
        "qx = np.tensordot(self.s[:, 1], self.e, axes=(0, 0))"),
    "greedy_strict_less": (
        "if dist <= delta:",
        "if dist < delta:"),
    "blackbody_corner_order": (
        "        if c.y_edge == BLACKBODY:\n            e[:, 0, :] = w * c.t_y_lo\n"
        "            e[:, c.ny - 1, :] = w * c.t_y_hi\n        if c.x_edge == BLACKBODY:\n"
        "            e[:, :, 0] = w * c.t_x_lo\n            e[:, :, c.nx - 1] = w * c.t_x_hi",
        "        if c.x_edge == BLACKBODY:\n            e[:, :, 0] = w * c.t_x_lo\n"
        "            e[:, :, c.nx - 1] = w * c.t_x_hi\n        if c.y_edge == BLACKBODY:\n"
        "            e[:, 0, :] = w * c.t_y_lo\n            e[:, c.ny - 1, :] = w * c.t_y_hi"),
    "specular_mirrors_wrong_axis": (
        "[self._find(d.sx, -d.sy) for d in self.dirs]",
        "[self._find(-d.sx, d.sy) for d in self.dirs]"),
    "specular_lands_one_row_in": (
        "new[j, 0, :] += p * lo",
        "new[j, 1, :] += p * lo"),
    "specular_share_also_diffused": (
        "r_lo += (1.0 - p) * lo",
        "r_lo += lo"),
    "corner_node_ignores_specularity": (
        "Tg[0] = (1.0 - c.y_specularity) * c.t_x_lo",
        "Tg[0] = c.t_x_lo"),
    "sources_before_blackbody": (
        "        self._apply_blackbody(new)\n        self._apply_sources(new)",
        "        self._apply_sources(new)\n        self._apply_blackbody(new)"),
    "speed_without_lead": (
        "r = speeds[i] * n + 1.0",
        "r = speeds[i] * (n + 1.0)"),
    "sources_not_imposed_at_start": (
        "        self._apply_blackbody(self.e)\n        self._apply_sources(self.e)",
        "        self._apply_blackbody(self.e)"),
}


def _load_mutant(name, old, new):
    with open(ORACLE) as f:
        src = f.read()
    assert src.count(old) == 1, f"snippet of {name} must occur exactly once"
    src = src.replace(old, new)
    modname = f"oracle_mutant_{name}"
    mod = types.ModuleType(modname)
    mod.__file__ = ORACLE
    sys.modules[modname] = mod
    try:
        exec(compile(src, ORACLE, "exec"), mod.__dict__)
    except Exception:
        del sys.modules[modname]
        raise
    return mod


def _consistency_checks(o):
    """Checks beyond the pins: the nearest-lattice-point form of the greedy
    (ties to the diagonal, from the '<=' of Eq. worm-paths) and the pull-form
    step matrix of every boundary combination."""
    saved = checks.o
    checks.o = o
    try:
        checks.test_worm_greedy_is_nearest_lattice_point()
        for xe, ye in [("blackbody", "blackbody"), ("periodic", "diffuse")]:
            checks.test_push_step_equals_pull_matrix(xe, ye, 16, "uniform")
    finally:
        checks.o = saved


def _wall_source_checks(o):
    """The specular-wall and source pins of test_oracle_walls_sources."""
    import test_oracle_walls_sources as wchecks
    saved = wchecks.o
    wchecks.o = o
    try:
        wchecks.test_specular_film_equals_mirrored_periodic_film(16, "uniform", "blackbody")
        wchecks.test_specular_diffuse_conserves_energy_and_keeps_equilibrium(0.35)
        wchecks.test_source_wins_over_blackbody_wall_and_is_imposed_at_start()
        wchecks.test_source_lays_values_along_worm_paths(16, "uniform")
        wchecks.test_axial_hop_count_closed_form(0.5)
        wchecks.test_slowed_axis_travels_at_its_speed()
    finally:
        wchecks.o = saved


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name):
    old, new = MUTATIONS[name]
    mod = _load_mutant(name, old, new)
    try:
        caught = []
        for pin in pins.ALL_PINS + [_consistency_checks, _wall_source_checks]:
            try:
                pin(mod)
            except Exception as exc:   # AssertionError or a crash of the mutant
                caught.append((pin.__name__, type(exc).__name__))
                break
        assert caught, f"mutation {name} passed every pin"
    finally:
        sys.modules.pop(f"oracle_mutant_{name}", None)


ADJOINT = os.path.join(os.path.dirname(ORACLE), "adjoint.py")

ADJOINT_MUTATIONS = {
    "walls_not_absorbed": (
        "        lam[:, wall] = 0.0",
        "        lam[:, wall] *= 1.0"),
    "eed_gradient_dropped": (
        "gW += -dd + e_prev.sum(axis=0) * G",
        "gW += -dd"),
    "adjoint_hops_on_pause": (
        "out[j] = (1.0 - W) * _pull(lam[j], hx, hy, c) + W * G",
        "out[j] = (1.0 - W) * _pull(lam[j], sx, sy, c) + W * G"),
    "adjoint_equilibrium_unweighted": (
        "G += lat.w[i] * _pull(lam[i], sx, sy, c)",
        "G += _pull(lam[i], sx, sy, c) / c.q"),
    "adjoint_pulls_from_wrong_side": (
        "return pad[1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]",
        "return pad[1 - dy:1 - dy + ny, 1 - dx:1 - dx + nx]"),
    "seed_without_factor_two": (
        "np.add.at(s, (py, px), 2.0 * d)",
        "np.add.at(s, (py, px), d)"),
    "mfp_chain_rule_wrong": (
        "dWc = f * (1.0 - 2.0 * Wp + 2.0 * Wp * lat.lam)",
        "dWc = f * (1.0 - Wp + Wp * lat.lam)"),
}


@pytest.mark.parametrize("name", sorted(ADJOINT_MUTATIONS))
def test_adjoint_mutation_is_caught(name):
    import test_oracle_adjoint as adj_checks
    old, new = ADJOINT_MUTATIONS[name]
    with open(ADJOINT) as f:
        src = f.read()
    assert src.count(old) == 1, f"snippet of {name} must occur exactly once"
    mod = types.ModuleType("oracle.adjoint_mutant")
    mod.__file__ = ADJOINT
    mod.__package__ = "oracle"
    exec(compile(src.replace(old, new), ADJOINT, "exec"), mod.__dict__)
    saved = adj_checks.adj
    adj_checks.adj = mod
    caught = False
    try:
        for args in [("blackbody", "blackbody", 16, "ring")]:
            try:
                adj_checks.test_transposed_step_equals_jacobian_transpose(*args)
            except Exception:
                caught = True
        for args in [("blackbody", "periodic", False, 16, "uniform"),
                     ("blackbody", "blackbody", True, 16, "uniform"),
                     ("periodic", "periodic", False, 24, "ring")]:
            if caught:
                break
            try:
                adj_checks.test_gradients_match_central_differences(*args)
            except Exception:
                caught = True
    finally:
        adj_checks.adj = saved
    assert caught, f"mutation {name} passed every adjoint pin"
