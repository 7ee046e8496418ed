"""MI355X-native sparse-grid hot path with AsyncTaichi's inter-kernel
optimizer (arXiv 2012.08141).

Modules: ``inputs`` (seeded workloads), ``grid`` (sparse grid handles),
``engine`` (tasks, run_sequence), ``programs`` (workload task programs).
The compute lives in ``libatsparse.so`` (HIP kernels for gfx950); importing
``grid``/``engine`` loads it and fails loudly if it is missing.
"""
__all__ = ["inputs", "grid", "engine", "programs"]
