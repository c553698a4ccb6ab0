"""Seeded synthetic problem descriptions shared by the oracle, tests and benchmark."""
from .workloads import *  # noqa: F401,F403
