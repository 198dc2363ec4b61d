"""The Sedov-Taylor reference that the point-blast GPU test is measured against."""
import pytest

import sedov_similarity as S


@pytest.mark.parametrize("gamma", [1.4, 5.0 / 3.0])
def test_similarity_solution_conserves_the_swept_mass(gamma):
    # the mass inside the shock equals the mass the shock has swept up: a check
    # of the integration that the equations do not impose directly
    assert S.mass_fraction(gamma) == pytest.approx(1.0, abs=1e-5)


def test_xi0_values():
    # the constant of R = xi0 (E t^2/rho0)^(1/5): about 1.03 for gamma = 1.4 and
    # about 1.15 for gamma = 5/3 in three dimensions
    assert S.xi0(1.4) == pytest.approx(1.0328, abs=2e-4)
    assert S.xi0(5.0 / 3.0) == pytest.approx(1.1517, abs=2e-4)
    assert S.radius(1.0, 1.4) == pytest.approx(S.xi0(1.4))
