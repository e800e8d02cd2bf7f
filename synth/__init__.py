"""Seeded synthetic OFDM massive-MIMO uplink frames.

This module is the transmitter and the channel: it draws bits, maps them to
QAM symbols, builds the frequency grid with comb pilots in symbol 0, passes it
through a seeded channel and synthesises complex64 time samples with additive
noise.  It holds none of the receiver's arithmetic (no FFT stage, no channel
estimation, no detection, no demapping) and imports neither the oracle nor
the HIP package; both consume what it produces.
"""
from .frames import (  # noqa: F401
    Shape, Frame, CONFIGS, STREAMS, config_shape, make_frame, make_frames,
    qam_map, used_bins, pilot_user, fft_framing, draw_batch_shapes, draw_inputs, quantize_sc16,
)
