"""Serving plumbing: one device arena owned by torch, requests handed to libtnc's server.

The server (C++, include/tnc.h) admits requests by HBM footprint, gives each admitted one a
stream and interleaves their slice batches on the device; this module only builds the
network handles, submits them and collects results.
"""

from __future__ import annotations

import numpy as np

from . import tnc
from .network import TensorNetwork


class Server:
    def __init__(self, arena_bytes: int, max_slots: int = 4, chunk_batches: int = 4,
                 device: int = 0):
        import torch
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=torch.device("cuda", device))
        self.device = device
        self._h = tnc.tnc_server_create(device, self.arena.data_ptr(), arena_bytes, max_slots,
                                        chunk_batches)
        self._shape = {}

    def submit(self, net: TensorNetwork, path, sliced_labels, slice_ids, open_qubits,
               closed_bits, n_samples: int = 0, seed: int = 0, precision: int = tnc.TNC_C64,
               max_batch_slices: int = 0) -> int:
        h = tnc.tnc_net_create(self.device, net.n_qubits, net.ranks(), net.flat_labels(),
                               net.flat_data(), net.out_label)
        try:
            tnc.tnc_net_set_path(h, path)
            tnc.set_slices_any(h, sliced_labels, slice_ids)
            tnc.tnc_net_set_targets(h, open_qubits, closed_bits)
            rid = tnc.tnc_server_submit(self._h, h, precision, max_batch_slices, n_samples, seed)
        finally:
            tnc.tnc_net_destroy(h)
        self._shape[rid] = (len(closed_bits), 1 << len(open_qubits), n_samples)
        return rid

    def poll(self, rid: int):
        """None while the request runs, else a dict with amplitudes, bitstrings and times;
        raises TncError with the request's status if it failed."""
        L, l, k = self._shape[rid]
        amps = np.zeros((L, l), dtype=np.complex128)
        bits = np.zeros(k, dtype=np.uint64) if k else None
        try:
            st, info = tnc.tnc_server_poll(self._h, rid, amps.view(np.float64), bits)
        except tnc.TncError:
            self._shape.pop(rid, None)     # the failed request is retired; its status raises
            raise
        if st == tnc.TNC_E_BUSY:
            return None
        del self._shape[rid]
        return {"amps": amps, "bits": bits, "t_submit": info.t_submit, "t_admit": info.t_admit,
                "t_done": info.t_done, "norm": info.norm, "slices": info.slices,
                "footprint": info.footprint_bytes}

    def pending(self):
        return tnc.tnc_server_pending(self._h)

    def close(self):
        if self._h is not None:
            tnc.tnc_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
