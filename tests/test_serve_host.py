"""Host logic of the server that needs no GPU: which of its classes a shot goes to."""
import types

import pytest

from paper_2504_06182_amd.pipeline import SIZE_CLASSES, size_class
from paper_2504_06182_amd.serve import Server, poisson_arrivals


def test_class_of_takes_the_smallest_class_that_holds_the_grid():
    srv = types.SimpleNamespace(classes={64: None, 128: None, 256: None})
    f = lambda shape: Server.class_of(srv, shape)
    assert f((32, 32, 5, 5, 27, 27)) == 64
    assert f((64, 48, 0, 0, 64, 48)) == 64
    assert f((96, 96, 14, 14, 81, 81)) == 128
    assert f((192, 192, 29, 29, 163, 163)) == 256      # no 192 class on this server
    with pytest.raises(ValueError):
        f((300, 300, 0, 0, 300, 300))


def test_launch_size_classes():
    assert SIZE_CLASSES == (64, 128, 192, 256)
    assert [size_class((s, s, 0, 0, s, s)) for s in (32, 64, 65, 128, 129, 192, 193, 256)] == \
        [64, 64, 128, 128, 192, 192, 256, 256]
    with pytest.raises(ValueError):
        size_class((257, 8, 0, 0, 1, 1))


def test_poisson_arrivals_seeded_and_in_range():
    a = poisson_arrivals(20000.0, 0.5, seed=50)
    assert len(a) > 9000 and len(a) < 11000 and a.min() >= 0 and a.max() < 0.5
    assert (a[1:] >= a[:-1]).all()
    assert (a == poisson_arrivals(20000.0, 0.5, seed=50)).all()
