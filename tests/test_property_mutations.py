"""The property checks of test_properties.py catch plausible mistakes: each
case plants one in a private copy of the oracle's C source (a sign in one
DMI neighbour direction, the anisotropy field booked under the dipolar
parameter, an exchange neighbour dropped, a wrong spin component in the
dipole sum), builds it, and requires at least one property to fail on it.
The oracle under oracle/ is not touched."""
import importlib.util
import os
import shutil

import pytest

import test_properties as tp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTATIONS = {
    "dmi_sign": ("h[0] += -d * (px[2] - mx[2]);", "h[0] += -d * (px[2] + mx[2]);"),
    "anisotropy_parameter": ("h[2] += 2.0 * k * sz[i];", "h[2] += 2.0 * D * sz[i];"),
    "exchange_neighbour": ("h[c] = J * (px[c] + mx[c] + py[c] + my[c] + pz[c] + mz[c]);",
                           "h[c] = J * (px[c] + mx[c] + py[c] + my[c] + pz[c]);"),
    "dipole_component": ("ay += 3.0 * ry * rs / r5 - sy[jj] / r3;", "ay += 3.0 * ry * rs / r5 - sx[jj] / r3;"),
}

PROPERTIES = ["test_field_operator_is_symmetric", "test_field_is_linear_in_the_spins",
              "test_energy_is_linear_in_the_parameters", "test_energy_is_minus_half_s_dot_h"]


def mutated_oracle(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site not found: " + name
    d = tmp_path / name
    d.mkdir()
    (d / "oracle.c").write_text(src.replace(old, new))
    shutil.copy(os.path.join(ROOT, "oracle", "oracle.py"), d / "oracle.py")
    spec = importlib.util.spec_from_file_location("oracle_mut_" + name, str(d / "oracle.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    m.build(force=True)
    return m


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(tmp_path, name):
    m = mutated_oracle(tmp_path, name, *MUTATIONS[name])
    for prop in PROPERTIES:
        try:
            getattr(tp, prop)(oracle=m)
        except AssertionError:
            return
    pytest.fail(name + " passed every property")


def test_unmutated_copy_passes(tmp_path, oracle):
    """The same harness on an unchanged copy passes every property."""
    m = mutated_oracle(tmp_path, "none", "double h[3];", "double h[3];")
    for prop in PROPERTIES:
        getattr(tp, prop)(oracle=m)
