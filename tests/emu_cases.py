"""Seeded cases shared by the CPU pins of the step emulator and the GPU
bit-level tests: a ragged gradient generator whose valves switch every few
steps (inlets, outlets, closed valves, walls), a periodic obstacle mask with
a source patch and first-order decay, and the straight channel started on
its developed Poiseuille state."""
import numpy as np

from paper_1307_4703_amd import workloads as W


def cases():
    out = {}
    out["gradient_generator"] = (W.gradient_generator(nx=300, ny=150, half_period=5,
                                                      peclet=300.0), None)
    m = W.random_mask(131, 67, seed=3, periodic=(True, False))
    wl = W.Workload("random_source_decay", m, tau_f=0.7, D=0.02, k_decay=2e-3,
                    periodic=(True, False))
    R = np.zeros(m.shape)
    rng = np.random.default_rng(17)
    R[20:36, 40:70] = 1e-3 * rng.random((16, 30))
    out["random_source_decay"] = (wl, R)
    out["straight_channel"] = (W.straight_channel(96, 40), None)
    return out
