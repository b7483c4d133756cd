"""FP64 reference of the converted feed-forward network of integrate-and-fire
neurons (ANN to SNN conversion section).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.  It shares no
code with the HIP path.

What is computed, for a batch of B images and T steps of dt = 1 ms:

- the input layer is analog: pixel p enters as x = p / 255, the same value at
  every step (the image is presented as a constant real-valued input);
- each hidden layer l is made of non-leaky IF neurons with reset by
  subtraction: at every step its voltage gains the input current
  I = a_{l-1} W_l + b_l (a_0 = x, a_l = the 0/1 spikes of layer l in the same
  step); a neuron whose voltage reaches the threshold theta_l spikes and has
  theta_l subtracted, so the excess above threshold is kept;
- the input of the output layer, s_L W_out + b_out, is summed over the run,
  and the predicted class is the index of the largest sum (the first one on a
  tie).

Readings where the text is silent (each listed with its reason in the design
notes): the analog input; the same-step propagation through the layers (the
table of accuracy against simulation time has above-chance accuracy after one
step, which a delay per layer would not allow); at most one spike per neuron
and step; voltages start at 0 in every run and have no lower bound; biases
enter as a constant current at every step.  The output layer's own spikes do
not affect the readout and are not simulated.
"""
from __future__ import annotations

import numpy as np


def if_step(v: np.ndarray, current: np.ndarray, theta: float):
    """One step of IF neurons with reset by subtraction (ANN to SNN
    conversion section): integrate, compare with the threshold, subtract the
    threshold from the neurons that spiked.  Returns (voltage after the step,
    voltage before the reset, spikes)."""
    u = v + current
    s = u >= theta
    return u - theta * s, u, s


class OracleIFNet:
    """The converted network: ``layers`` = [(W_1, b_1), ..., (W_out, b_out)]
    with W_l of shape (n_{l-1}, n_l); ``thresholds`` one per hidden layer."""

    def __init__(self, layers, thresholds):
        self.layers = [(np.asarray(W, np.float64), np.asarray(b, np.float64)) for W, b in layers]
        self.thresholds = [float(t) for t in thresholds]
        assert len(self.thresholds) == len(self.layers) - 1
        for (Wa, _), (Wb, _) in zip(self.layers, self.layers[1:]):
            assert Wa.shape[1] == Wb.shape[0]

    def run(self, images: np.ndarray, T: int, record=()) -> dict:
        """Simulate ``images`` (B, n_in) uint8 for T steps from rest.

        Always returns ``out`` (B, n_out) summed output-layer input and
        ``pred`` (B,) its argmax.  ``record`` may add, per hidden layer l
        (1-based): ``s{l}`` (B, T, n_l) uint8 spikes, ``v{l}`` (B, T, n_l)
        voltage after each step, ``u{l}`` (B, T, n_l) voltage before the
        reset (after integration), ``c{l}`` (B, n_l) spike counts."""
        x = np.asarray(images, np.float64) / 255.0
        B = x.shape[0]
        hidden = self.layers[:-1]
        W_out, b_out = self.layers[-1]
        v = [np.zeros((B, W.shape[1])) for W, _ in hidden]
        res = {}
        for l, (W, _) in enumerate(hidden, start=1):
            n = W.shape[1]
            if f"s{l}" in record:
                res[f"s{l}"] = np.zeros((B, T, n), np.uint8)
            for key in ("v", "u"):
                if f"{key}{l}" in record:
                    res[f"{key}{l}"] = np.zeros((B, T, n))
            if f"c{l}" in record:
                res[f"c{l}"] = np.zeros((B, n), np.int64)
        out = np.zeros((B, W_out.shape[1]))
        for t in range(T):
            a = x
            for l, ((W, b), th) in enumerate(zip(hidden, self.thresholds), start=1):
                v[l - 1], u, s = if_step(v[l - 1], a @ W + b, th)
                if f"s{l}" in res:
                    res[f"s{l}"][:, t] = s
                if f"v{l}" in res:
                    res[f"v{l}"][:, t] = v[l - 1]
                if f"u{l}" in res:
                    res[f"u{l}"][:, t] = u
                if f"c{l}" in res:
                    res[f"c{l}"] += s
                a = s.astype(np.float64)
            out += a @ W_out + b_out
        res["out"] = out
        res["pred"] = np.argmax(out, axis=1)
        return res


def ann_forward(layers, images: np.ndarray) -> list:
    """Activations of the ReLU network the IF network approximates (the same
    weights, ReLU instead of spiking): [a_1, ..., a_{L-1}, output]."""
    a = np.asarray(images, np.float64) / 255.0
    acts = []
    for l, (W, b) in enumerate(layers):
        z = a @ np.asarray(W, np.float64) + np.asarray(b, np.float64)
        a = z if l == len(layers) - 1 else np.maximum(z, 0.0)
        acts.append(a)
    return acts
