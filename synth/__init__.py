"""Seeded synthetic input generators (no method arithmetic)."""
from .generators import (V_MASK, WORKLOADS, Workload, cube_on_device, data_events,
                         down_events, epoch_permutations,
                         event_cube, make_problem, model_draw, onsets, positions, random_arrays,
                         random_batch, random_onsets,
                         reflection_events, ricker, scale_noise, streams, vs_positions)

__all__ = ["V_MASK", "WORKLOADS", "Workload", "cube_on_device", "data_events",
           "down_events", "epoch_permutations",
           "event_cube", "make_problem", "model_draw", "onsets", "positions",
           "random_arrays", "random_batch", "random_onsets",
           "reflection_events", "ricker", "scale_noise", "streams", "vs_positions"]
