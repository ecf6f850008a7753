"""Cached problem builds shared by the tests (inputs only)."""
import functools

from fixture.problem import build_problem


@functools.lru_cache(maxsize=None)
def problem(name, nsteps=None):
    return build_problem(name, nsteps=nsteps)


@functools.lru_cache(maxsize=None)
def oracle(name, nsteps=None):
    from oracle.mot_oracle import Oracle
    return Oracle(problem(name, nsteps))
