"""Seeded workloads shared by the tests of one process (building the larger
ones takes up to a minute on the host, so each is built once)."""
import functools

import synth


@functools.lru_cache(maxsize=None)
def config(k: int):
    """synth.config(k), built once per test process (callers must not modify
    the arrays; dataclasses.replace makes a modified copy)."""
    return synth.config(k)
