"""The oracle against its pins (CPU only): the single-thread build and the all-cores (OpenMP) build of
the same source each pass every pin."""
import pytest

import oracle
import pins


@pytest.fixture(scope="module", params=["one thread", "all cores"])
def orc(request):
    if request.param == "one thread":
        oracle.build()
        return oracle.Oracle()
    return oracle.get_all_cores()


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(orc, pin):
    pin(orc)
