"""MI355X-native bosonic PIMD exchange potential and forces (quadratic-scaling
algorithm of Feldman & Hirshberg).

    from paper_2305_18025_amd import BosonicExchange, exchange_potential

The compute path is libpimdb.so (HIP, gfx950), built by
``paper_2305_18025_amd.build``; this package only marshals arguments.
"""
from .core import BosonicExchange  # noqa: F401
from .autograd import exchange_potential  # noqa: F401
from .md import VelocityVerlet  # noqa: F401
from . import inputs  # noqa: F401

__all__ = ["BosonicExchange", "exchange_potential", "VelocityVerlet", "inputs"]
