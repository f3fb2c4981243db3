"""Host-side argument checks of the DOS / LDOS module (no GPU)."""
import numpy as np
import pytest

from paper_1405_0194_amd import dos as pdos


@pytest.mark.parametrize("edges", [np.array([0.0]), np.array([0.0, 0.0]), np.array([0.1, 0.0]),
                                   np.zeros((2, 2))])
def test_dos_rejects_bad_edges(edges):
    with pytest.raises(ValueError):
        pdos.dos(None, None, None, edges)


def test_ldos_rejects_nonpositive_eta():
    with pytest.raises(ValueError):
        pdos.ldos(None, None, None, np.array([0.0]), 0.0)
