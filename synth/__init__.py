"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

This package holds only workload descriptions and raw random draws (positions,
noise scales, standard-normal deviates).  It contains none of the method's
arithmetic: the prior draw of the true field and the line-of-sight extinction
of each star are computed separately by the oracle and by the GPU library from
the deviates drawn here.
"""
from .workloads import Workload, preset, draw, gmm_catalogue, PRESETS  # noqa: F401
