"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package produces only *inputs* of the F-statistic search: the detector
ephemeris (the content of the paper's detector-to-SSB file), Gaussian noise,
injected continuous-wave signals, and template lists (sky positions and
spindowns).  It contains none of the search's own arithmetic: the injected
signal's antenna response is evaluated from the detector tensor, not from the
closed-form amplitude modulations the search uses.
"""
from .inputs import *  # noqa: F401,F403
