"""Measurement programs beside bench.py: per-size tables of the paper's problems, precision and
uneven-size runs, conjugate-gradient runs, and rocprofv3 helpers.  Run as
``python -m benchmarks.<name>`` from the repository root."""
