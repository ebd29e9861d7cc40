"""Seeded synthetic inputs shared by the checker, the tests and the benchmark.

Holds scene definitions only (lighting, frames, transport in the pixel domain);
none of the method's arithmetic lives here."""
from .scene import *  # noqa: F401,F403
from .scene import WORKLOADS, Workload  # noqa: F401
