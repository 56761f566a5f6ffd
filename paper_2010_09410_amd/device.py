"""torch-facing wrapper of libvsp: device buffers are torch tensors, streams are torch streams.

Torus arrays live on the device as int32 tensors holding the uint32 bit patterns; the
helpers below convert from and to numpy uint32. Every call goes through the C ABI in
``_native``; nothing here computes on ciphertexts.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _native as nv


def to_device(arr, device) -> torch.Tensor:
    a = np.ascontiguousarray(arr)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).to(device)


def to_host(t: torch.Tensor) -> np.ndarray:
    a = t.detach().cpu().numpy()
    return a.view(np.uint32) if a.dtype == np.int32 else a


def _ptr(t: torch.Tensor) -> int:
    assert t.is_contiguous(), "tensors passed to libvsp must be contiguous"
    return t.data_ptr()


class Context:
    """A libvsp context on one GPU: keys resident in device memory (Bob's evaluation keys)."""

    N_LWE, N_RING, L = 630, 1024, 3

    def __init__(self, bk: np.ndarray, ksk: np.ndarray, device: int = 0):
        self.device = torch.device("cuda", device)
        torch.cuda.set_device(self.device)
        self.handle = nv.vsp_context_create(np.ascontiguousarray(bk, dtype=np.uint32),
                                            np.ascontiguousarray(ksk, dtype=np.uint32), device)

    # -------------------------------------------------------------- lifecycle
    def close(self) -> None:
        if getattr(self, "handle", None):
            nv.vsp_context_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def stream(self):
        return torch.cuda.current_stream(self.device).cuda_stream

    def sync(self) -> None:
        nv.vsp_context_sync(self.handle)

    def tensor(self, arr) -> torch.Tensor:
        return to_device(arr, self.device)

    def empty(self, *shape) -> torch.Tensor:
        return torch.empty(shape, dtype=torch.int32, device=self.device)

    # -------------------------------------------------------------- gates
    def gates(self, ops: torch.Tensor, in0: torch.Tensor, in1: torch.Tensor, mode: int = nv.VSP_BATCHED,
              out: torch.Tensor | None = None) -> torch.Tensor:
        B = ops.numel()
        if out is None:
            out = self.empty(B, self.N_LWE + 1)
        nv.vsp_gates(self.handle, _ptr(ops), _ptr(in0), _ptr(in1), _ptr(out), B, mode, self.stream())
        return out

    def gates_key_copies(self, ops, in0, in1, waves: int, copies: int, out=None):
        """(outputs, blind-rotation ms) of gates whose gate g reads its own key copy g mod copies."""
        B = ops.numel()
        if out is None:
            out = self.empty(B, self.N_LWE + 1)
        ms = nv.vsp_gates_key_copies(self.handle, _ptr(ops), _ptr(in0), _ptr(in1), _ptr(out), B, waves, copies,
                                     self.stream())
        return out, ms

    def mux(self, sel: torch.Tensor, in1: torch.Tensor, in0: torch.Tensor, out=None) -> torch.Tensor:
        """Encrypted sel ? in1 : in0, row by row."""
        B = sel.shape[0]
        if out is None:
            out = self.empty(B, self.N_LWE + 1)
        nv.vsp_mux(self.handle, _ptr(sel), _ptr(in1), _ptr(in0), _ptr(out), B, self.stream())
        return out

    def bootstrap_trlwe(self, ops, in0, in1, out=None) -> torch.Tensor:
        B = ops.numel()
        if out is None:
            out = self.empty(B, 2, self.N_RING)
        nv.vsp_bootstrap_trlwe(self.handle, _ptr(ops), _ptr(in0), _ptr(in1), _ptr(out), B, self.stream())
        return out

    # -------------------------------------------------------------- CMUX memory
    def rom_read(self, rom: torch.Tensor, addr: torch.Tensor, v: int, w: int, out=None) -> torch.Tensor:
        R = addr.shape[0]
        if out is None:
            out = self.empty(R, w, self.N_LWE + 1)
        nv.vsp_rom_read(self.handle, _ptr(rom), rom.shape[0], _ptr(addr), v, w, _ptr(out), R, self.stream())
        return out

    def ram_read(self, ram: torch.Tensor, addr: torch.Tensor, out=None) -> torch.Tensor:
        w, cells = ram.shape[0], ram.shape[1]
        v = int(cells).bit_length() - 1
        R = addr.shape[0]
        if out is None:
            out = self.empty(R, w, self.N_LWE + 1)
        nv.vsp_ram_read(self.handle, _ptr(ram), v, w, _ptr(addr), _ptr(out), R, self.stream())
        return out

    def ram_write(self, ram: torch.Tensor, addr: torch.Tensor, flag: torch.Tensor, data: torch.Tensor) -> None:
        w, cells = ram.shape[0], ram.shape[1]
        v = int(cells).bit_length() - 1
        nv.vsp_ram_write(self.handle, _ptr(ram), v, w, _ptr(addr), _ptr(flag), _ptr(data), self.stream())

    # -------------------------------------------------------------- launch tuning
    def autotune(self, max_batch: int = 4096, cache_path: str | None = None) -> None:
        nv.vsp_autotune(self.handle, max_batch, cache_path)

    def tuning(self, B: int):
        return nv.vsp_tuning_get(self.handle, B)

    def set_tuning(self, B: int, br_waves: int, ks_form: int) -> None:
        nv.vsp_tuning_set(self.handle, B, br_waves, ks_form)

    def set_split_groups(self, B: int, groups: int) -> int:
        return nv.vsp_tuning_set_split(self.handle, B, groups)

    # -------------------------------------------------------------- circuits / serving
    def circuit(self, gates, ninputs: int) -> "Circuit":
        return Circuit(self, gates, ninputs)

    def machine(self, gates, ninputs: int, next_state) -> "Machine":
        return Machine(self, gates, ninputs, next_state)

    def keyset(self, bk: np.ndarray, ksk: np.ndarray) -> "Keyset":
        return Keyset(self, bk, ksk)

    def cbkey(self, bk2: np.ndarray, pksk: np.ndarray) -> "CbKey":
        return CbKey(self, bk2, pksk)

    def server(self, mem_budget_bytes: int, max_batch: int = 4096) -> "Server":
        return Server(self, mem_budget_bytes, max_batch)

    # -------------------------------------------------------------- test entries
    def debug_external_product(self, C: torch.Tensor, x: torch.Tensor, out=None) -> torch.Tensor:
        J = C.shape[0]
        if out is None:
            out = self.empty(J, 2, self.N_RING)
        nv.vsp_debug_external_product(self.handle, _ptr(C), _ptr(x), _ptr(out), J, self.stream())
        return out

    def debug_polymul(self, a: torch.Tensor, b: torch.Tensor, out=None) -> torch.Tensor:
        J = a.shape[0]
        if out is None:
            out = self.empty(J, self.N_RING)
        nv.vsp_debug_polymul(self.handle, _ptr(a), _ptr(b), _ptr(out), J, self.stream())
        return out


class Circuit:
    """A levelled circuit captured for replay (HIP graph of one batched launch per level)."""

    def __init__(self, ctx: Context, gates, ninputs: int):
        self.ctx = ctx
        self.gates = np.asarray(gates, dtype=np.int64)
        self.ninputs = int(ninputs)
        self.handle = nv.vsp_circuit_create(ctx.handle, self.gates, self.ninputs)
        self.nlevels, self.max_width = nv.vsp_circuit_info(self.handle)

    @property
    def nwires(self) -> int:
        return self.ninputs + len(self.gates)

    def run(self, inputs: torch.Tensor, wires: torch.Tensor | None = None) -> torch.Tensor:
        if wires is None:
            wires = self.ctx.empty(self.nwires, self.ctx.N_LWE + 1)
        nv.vsp_circuit_run(self.handle, _ptr(inputs), _ptr(wires), self.ctx.stream())
        return wires

    def run_timed(self, inputs: torch.Tensor, wires: torch.Tensor | None = None):
        if wires is None:
            wires = self.ctx.empty(self.nwires, self.ctx.N_LWE + 1)
        ms = nv.vsp_circuit_run_timed(self.handle, _ptr(inputs), _ptr(wires), self.ctx.stream(), self.nlevels)
        return wires, ms

    def close(self) -> None:
        if getattr(self, "handle", None):
            nv.vsp_circuit_destroy(self.handle)
            self.handle = None


class Machine:
    """A clocked circuit: external inputs, flip-flops latching named wires every cycle, and a
    levelled gate DAG replayed as one HIP graph per cycle."""

    def __init__(self, ctx: Context, gates, ninputs: int, next_state):
        self.ctx = ctx
        self.gates = np.asarray(gates, dtype=np.int64)
        self.ninputs = int(ninputs)
        self.nstate = int(np.asarray(next_state).size)
        self.handle = nv.vsp_machine_create(ctx.handle, self.gates, self.ninputs, next_state)

    @property
    def nwires(self) -> int:
        return self.ninputs + self.nstate + len(self.gates)

    def run(self, state: torch.Tensor, ncycles: int, inputs: torch.Tensor | None = None,
            wires: torch.Tensor | None = None) -> torch.Tensor:
        """Advances `state` ([nstate][n+1], updated in place) by ncycles cycles; inputs are
        [ncycles][ninputs][n+1]. Returns `wires` (all wires of the last cycle) if given."""
        nv.vsp_machine_run(self.handle, None if inputs is None else _ptr(inputs), _ptr(state),
                           None if wires is None else _ptr(wires), int(ncycles), self.ctx.stream())
        return wires

    def attach_ram(self, key: "CbKey", ram: torch.Tensor, addr_wires, flag_wire: int, data_wires, read_state) -> None:
        """RAM port: ram [w][2^v][2][N] (kept by the caller), updated every cycle."""
        w, cells = ram.shape[0], ram.shape[1]
        v = int(cells).bit_length() - 1
        self.ram = ram
        nv.vsp_machine_attach_ram(self.handle, key.handle, _ptr(ram), v, w, addr_wires, int(flag_wire), data_wires,
                                  read_state)

    def close(self) -> None:
        if getattr(self, "handle", None):
            nv.vsp_machine_destroy(self.handle)
            self.handle = None


class CbKey:
    """Circuit-bootstrapping keys on the context's GPU: level-2 bootstrapping key and the
    private key-switching keys."""

    def __init__(self, ctx: Context, bk2: np.ndarray, pksk: np.ndarray):
        self.ctx = ctx
        self.handle = nv.vsp_cbkey_create(ctx.handle, np.ascontiguousarray(bk2, dtype=np.uint64),
                                          np.ascontiguousarray(pksk, dtype=np.uint32))

    def set_form(self, form: int) -> None:
        """Level-2 blind rotation: 0 by batch size, 1 four-wave form, 2 eight-wave form."""
        nv.vsp_cbkey_set_form(self.handle, form)

    def bootstrap(self, tlwe: torch.Tensor, out=None) -> torch.Tensor:
        """TLWE [R][n+1] -> TRGSW [R][2l][2][N]."""
        R = tlwe.shape[0]
        if out is None:
            out = self.ctx.empty(R, 6, 2, 1024)
        nv.vsp_circuit_bootstrap(self.ctx.handle, self.handle, _ptr(tlwe), _ptr(out), R, self.ctx.stream())
        return out

    def close(self) -> None:
        if getattr(self, "handle", None):
            nv.vsp_cbkey_destroy(self.handle)
            self.handle = None


class Keyset:
    """Another client's bootstrapping and key-switching keys on the context's GPU."""

    def __init__(self, ctx: Context, bk: np.ndarray, ksk: np.ndarray):
        self.ctx = ctx
        self.handle = nv.vsp_keyset_create(ctx.handle, np.ascontiguousarray(bk, dtype=np.uint32),
                                           np.ascontiguousarray(ksk, dtype=np.uint32))

    def close(self) -> None:
        if getattr(self, "handle", None):
            nv.vsp_keyset_destroy(self.handle)
            self.handle = None


class Server:
    """Continuous-batching evaluation of many clients' circuits on one context."""

    def __init__(self, ctx: Context, mem_budget_bytes: int, max_batch: int):
        self.ctx = ctx
        self.handle = nv.vsp_server_create(ctx.handle, int(mem_budget_bytes), int(max_batch))

    def submit(self, gates, ninputs: int, inputs: np.ndarray, keyset: "Keyset | None" = None) -> int:
        gates = np.asarray(gates, dtype=np.int64)
        inputs = np.ascontiguousarray(inputs, dtype=np.uint32)
        if keyset is None:
            return nv.vsp_server_submit(self.handle, gates, int(ninputs), inputs)
        return nv.vsp_server_submit_keyset(self.handle, keyset.handle, gates, int(ninputs), inputs)

    def poll(self, ticket: int, nwires: int | None = None):
        """Returns (done, wires or None, latency_ms)."""
        buf = None if nwires is None else np.zeros((nwires, self.ctx.N_LWE + 1), dtype=np.uint32)
        done, lat = nv.vsp_server_poll(self.handle, ticket, buf)
        return done, (buf if done else None), lat

    def stats(self):
        return nv.vsp_server_stats(self.handle)

    def close(self) -> None:
        if getattr(self, "handle", None):
            nv.vsp_server_destroy(self.handle)
            self.handle = None
