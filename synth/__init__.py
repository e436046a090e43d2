"""Seeded synthetic inputs for the FLD solve (shared by the tests, the oracle
checks and the benchmark).  This package generates media only; it holds none
of the solver's arithmetic."""
from .media import (  # noqa: F401
    point_source,
    value_noise,
    cloud_extinction,
    beer_lambert_source,
    cloud_medium,
    config,
    batch_config,
    CONFIGS,
)
