"""A compiled contraction on one GPU, with torch providing the device memory.

Thin plumbing over the C ABI: the network, path, slices and targets are handed to
libtnc once; the workspace and the FP64 amplitude buffer are torch tensors whose raw
pointers the library writes.  Nothing here computes amplitudes.
"""

from __future__ import annotations

import numpy as np

from . import tnc
from .network import TensorNetwork


class Contraction:
    def __init__(self, net: TensorNetwork, path, sliced_labels=(), slice_ids=None,
                 open_qubits=(), closed_bits=(0,), precision: int = tnc.TNC_C64,
                 device: int = 0, max_batch_slices: int = 1):
        """max_batch_slices: slices per launch sequence; 0 lets the library choose."""
        import torch

        self.device = device
        self.n_qubits = net.n_qubits
        self.open_qubits = [int(q) for q in open_qubits]
        self.closed_bits = np.asarray(closed_bits, dtype=np.uint64)
        self.sliced_labels = [int(x) for x in sliced_labels]
        if slice_ids is None:
            slice_ids = np.arange(1 << len(self.sliced_labels), dtype=np.uint64)
        # more than 63 sliced labels: ids are Python ints of up to 127 bits
        self.slice_ids = (np.asarray(slice_ids, dtype=np.uint64) if len(self.sliced_labels) <= 63
                          else [int(x) for x in slice_ids])
        self._net = tnc.tnc_net_create(device, net.n_qubits, net.ranks(), net.flat_labels(),
                                       net.flat_data(), net.out_label)
        self._plan = None
        try:
            tnc.tnc_net_set_path(self._net, path)
            tnc.set_slices_any(self._net, self.sliced_labels, self.slice_ids)
            tnc.tnc_net_set_targets(self._net, self.open_qubits, self.closed_bits)
            self._plan = tnc.tnc_plan_create(self._net, precision, max_batch_slices)
        except Exception:
            self.close()
            raise
        self.ws_bytes = tnc.tnc_plan_workspace_bytes(self._plan)
        self.batch_slices = tnc.tnc_plan_batch_slices(self._plan)
        dev = torch.device("cuda", device)
        self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=dev)
        L, l = len(self.closed_bits), 1 << len(self.open_qubits)
        self.amps = torch.zeros((L, l), dtype=torch.complex128, device=dev)

    # -- calls ---------------------------------------------------------------------------
    @staticmethod
    def _stream(stream):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        return s.cuda_stream

    def contract(self, norm: bool = False, stream=None):
        return tnc.tnc_contract(self._plan, self.ws.data_ptr(), self.ws_bytes,
                                self._stream(stream), self.amps.data_ptr(), want_norm=norm)

    def contract_range(self, first: int, count: int, accumulate: bool = False, stream=None):
        tnc.tnc_contract_range(self._plan, self.ws.data_ptr(), self.ws_bytes,
                               self._stream(stream), self.amps.data_ptr(), first, count,
                               accumulate)

    def sample(self, seed: int, n_samples: int, stream=None) -> np.ndarray:
        return tnc.tnc_sample(self._plan, self.ws.data_ptr(), self.ws_bytes,
                              self.amps.data_ptr(), seed, n_samples, self._stream(stream))

    def sample_metropolis(self, seed: int, n_samples: int, steps: int, stream=None) -> np.ndarray:
        """In-group Metropolis chains of `steps` moves (one draw per chain)."""
        return tnc.tnc_sample_metropolis(self._plan, self.ws.data_ptr(), self.ws_bytes,
                                         self.amps.data_ptr(), seed, n_samples, steps,
                                         self._stream(stream))

    def sample_frugal(self, seed: int, n_samples: int, m: float = 10.0, max_trials: int = 64,
                      stream=None) -> np.ndarray:
        """Frugal rejection sampling with bound m and at most max_trials proposals."""
        return tnc.tnc_sample_frugal(self._plan, self.ws.data_ptr(), self.ws_bytes,
                                     self.amps.data_ptr(), seed, n_samples, m, max_trials,
                                     self._stream(stream))

    def autotune(self, reps: int = 3, stream=None) -> int:
        """Pick tile configurations and split-K per GEMM by timing them; returns how many
        launches changed."""
        return tnc.tnc_plan_autotune(self._plan, self.ws.data_ptr(), self.ws_bytes,
                                     self._stream(stream), reps)

    def stats(self):
        return tnc.tnc_plan_stats(self._plan)

    def work(self, first: int = 0, count: int | None = None) -> float:
        """Algorithmic flops contracting slices [first, first + count) executes (steps
        shared by a batch counted once per batch)."""
        n = len(self.slice_ids) - first if count is None else count
        return tnc.tnc_plan_work(self._plan, first, n)

    def launches(self):
        return [tnc.tnc_plan_launch_info(self._plan, i)
                for i in range(tnc.tnc_plan_n_launches(self._plan))]

    def set_timing(self, enable: bool):
        tnc.tnc_plan_set_timing(self._plan, enable)

    def timing(self, reset: bool = False):
        return tnc.tnc_plan_timing(self._plan, reset)

    def launch_timing(self):
        """(ms, count) per launch index since the last timing reset."""
        return [tnc.tnc_plan_launch_timing(self._plan, i)
                for i in range(tnc.tnc_plan_n_launches(self._plan))]

    def close(self):
        if self._plan is not None:
            tnc.tnc_plan_destroy(self._plan)
            self._plan = None
        if self._net is not None:
            tnc.tnc_net_destroy(self._net)
            self._net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
