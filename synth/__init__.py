"""Seeded synthetic RGB-D inputs shared by the oracle side and the HIP side."""
from .scenes import *  # noqa: F401,F403
