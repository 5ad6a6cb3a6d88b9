"""Seeded synthetic inputs (initial conditions) shared by the GPU library's
tests and benchmark and by the CPU oracle.  No solver arithmetic lives here."""
from . import problems  # noqa: F401
