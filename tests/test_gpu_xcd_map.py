"""The XCD mapping of the single-box edge and update passes only permutes
which workgroup takes which tile: the contiguous mapping (each XCD a
contiguous range of tiles) and the banded one (all XCDs on bands of the same
plane, the automatic choice for large planes) give the same step bit for
bit.  Every reconstruction and EMF scheme, both forms, with and without
resistivity, on ragged and degenerate boxes whose chunks end part-way."""
import numpy as np
import pytest

from paper_2609_10816_amd import ctmhd, inputs

pytestmark = pytest.mark.gpu


def _run(xcd_map, recon, emf, precision, eta, cons, bf, dx, nsteps):
    P = ctmhd.make_params(recon=recon, emf=emf, eta=eta, precision=precision,
                          tile=ctmhd.make_tile(xcd_map=xcd_map))
    return ctmhd.run(P, cons, bf, dx, nsteps)


@pytest.mark.parametrize("shape", [(40, 36, 33), (33, 20, 18), (70, 9, 21), (13, 7, 5),
                                   (17, 1, 1), (1, 6, 10)])
@pytest.mark.parametrize("recon,emf", [("pc", "q26"), ("plm", "b25a"), ("ppm", "q26"),
                                       ("ppm", "fs18")])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_banded_equals_contiguous(shape, recon, emf, precision):
    if min(shape) > 4:
        cons, bf, info = inputs.turbulent_box(shape, mach=3.0, b0=(0.4, 0.2, -0.1),
                                              db_rms=0.2, seed_v=61, seed_a=62)
    else:
        cons, bf, info = inputs.fast_wave(shape, kvec=tuple(1 if s > 1 else 0 for s in shape),
                                          delta=1e-3)
    dx = [1.0 / s for s in shape]
    eta = 1e-3 if recon != "plm" else 0.0
    a = _run("contiguous", recon, emf, precision, eta, cons, bf, dx, 2)
    b = _run("banded", recon, emf, precision, eta, cons, bf, dx, 2)
    np.testing.assert_array_equal(a[2], b[2])
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_automatic_mapping_on_a_large_box():
    """The automatic choice bands a 200 x 200 plane; its step is the
    contiguous mapping's."""
    cons, bf, info = inputs.turbulent_box((200, 200, 72), mach=2.0, b0=(0.5, 0.0, 0.0),
                                          db_rms=0.3, seed_v=63, seed_a=64)
    dx = [1.0 / 200, 1.0 / 200, 1.0 / 72]
    a = _run("auto", "ppm", "q26", "fp64", 1e-3, cons, bf, dx, 1)
    b = _run("contiguous", "ppm", "q26", "fp64", 1e-3, cons, bf, dx, 1)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
