"""Seeded synthetic inputs (images, opaque-quadrant patterns, sensor read-out)."""
from .inputs import *  # noqa: F401,F403
