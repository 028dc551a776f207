"""Seeded synthetic mid-simulation states (re-exported from the generators)."""

from paper_2406_10661_amd.workloads import synthetic_state  # noqa: F401
