"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark."""
from .cells import (CellSpec, TINY, MID, LEARNED, LARGE, LARGE_GRID, GRID108, batched_specs, fft_size,
                    miller_sorted, place_atoms, random_dv, stream_rng)
