"""The oracle against closed forms, exact arithmetic, LAPACK and invariants."""

import pytest

import oracle_checks as oc


@pytest.mark.parametrize("check", oc.ALL_CHECKS, ids=lambda f: f.__name__)
def test_oracle_pin(check):
    check()
