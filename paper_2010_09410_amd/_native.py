"""ctypes binding of libvsp (include/vsp.h): the same entry points, argument marshalling only.

Device pointers are passed as integers (e.g. ``torch.Tensor.data_ptr()``), streams as
integers (``torch.cuda.current_stream().cuda_stream``) or None. A non-zero status raises
VspError carrying the library's message. There is no fallback: if libvsp.so is missing,
importing this module's functions raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvsp.so")

VSP_OK, VSP_E_ARG, VSP_E_PARAMS, VSP_E_NOMEM, VSP_E_HIP, VSP_E_STATE, VSP_E_CAPACITY = 0, -1, -2, -3, -4, -5, -6
VSP_BATCHED, VSP_PER_GATE = 0, 1
NAND, AND, OR, NOR, XOR, XNOR, ANDNOT, ORNOT, NOT = range(9)


class VspError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


class vsp_params(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint32) for k in ("n", "N", "k", "l", "bg_bits", "ks_t", "ks_basebit")]


class vsp_gate_desc(ctypes.Structure):
    _fields_ = [("op", ctypes.c_uint32), ("in0", ctypes.c_uint32), ("in1", ctypes.c_uint32)]


DEFAULT_PARAMS = (630, 1024, 1, 3, 6, 8, 2)

_lib = None
_c = ctypes
_vp = ctypes.c_void_p
_u64 = ctypes.c_uint64
_i32 = ctypes.c_int
_st = ctypes.c_int32

SIGNATURES = {
    "vsp_status_str": (ctypes.c_char_p, [_st]),
    "vsp_last_error": (ctypes.c_char_p, []),
    "vsp_context_create": (_st, [ctypes.POINTER(vsp_params), _vp, _vp, _i32, ctypes.POINTER(_vp)]),
    "vsp_context_destroy": (_st, [_vp]),
    "vsp_context_sync": (_st, [_vp]),
    "vsp_gates": (_st, [_vp, _vp, _vp, _vp, _vp, _u64, _i32, _vp]),
    "vsp_gates_noalloc": (_st, [_vp, _vp, _vp, _vp, _vp, _u64, _i32, _vp]),
    "vsp_gates_key_copies": (_st, [_vp, _vp, _vp, _vp, _vp, _u64, _i32, ctypes.c_uint32, _vp,
                                   ctypes.POINTER(ctypes.c_double)]),
    "vsp_bootstrap_trlwe": (_st, [_vp, _vp, _vp, _vp, _vp, _u64, _vp]),
    "vsp_circuit_create": (_st, [_vp, ctypes.POINTER(vsp_gate_desc), _u64, _u64, ctypes.POINTER(_vp)]),
    "vsp_circuit_run": (_st, [_vp, _vp, _vp, _vp]),
    "vsp_circuit_run_timed": (_st, [_vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_float)]),
    "vsp_circuit_info": (_st, [_vp, ctypes.POINTER(_u64), ctypes.POINTER(_u64)]),
    "vsp_circuit_destroy": (_st, [_vp]),
    "vsp_rom_read": (_st, [_vp, _vp, ctypes.c_uint32, _vp, ctypes.c_uint32, ctypes.c_uint32, _vp, _u64, _vp]),
    "vsp_ram_read": (_st, [_vp, _vp, ctypes.c_uint32, ctypes.c_uint32, _vp, _vp, _u64, _vp]),
    "vsp_ram_write": (_st, [_vp, _vp, ctypes.c_uint32, ctypes.c_uint32, _vp, _vp, _vp, _vp]),
    "vsp_server_create": (_st, [_vp, _u64, _u64, ctypes.POINTER(_vp)]),
    "vsp_server_submit": (_st, [_vp, ctypes.POINTER(vsp_gate_desc), _u64, _u64, _vp, ctypes.POINTER(_u64)]),
    "vsp_server_poll": (_st, [_vp, _u64, _vp, ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_double)]),
    "vsp_server_stats": (_st, [_vp, ctypes.POINTER(_u64), ctypes.POINTER(_u64), ctypes.POINTER(_u64)]),
    "vsp_server_destroy": (_st, [_vp]),
    "vsp_machine_create": (_st, [_vp, ctypes.POINTER(vsp_gate_desc), _u64, _u64, _u64, _vp, ctypes.POINTER(_vp)]),
    "vsp_machine_run": (_st, [_vp, _vp, _vp, _vp, _u64, _vp]),
    "vsp_machine_destroy": (_st, [_vp]),
    "vsp_keyset_create": (_st, [_vp, _vp, _vp, ctypes.POINTER(_vp)]),
    "vsp_keyset_destroy": (_st, [_vp]),
    "vsp_cbkey_create": (_st, [_vp, _vp, _vp, ctypes.POINTER(_vp)]),
    "vsp_machine_attach_ram": (_st, [_vp, _vp, _vp, ctypes.c_uint32, ctypes.c_uint32, _vp, ctypes.c_uint32, _vp, _vp]),
    "vsp_cbkey_destroy": (_st, [_vp]),
    "vsp_cbkey_set_form": (_st, [_vp, _i32]),
    "vsp_circuit_bootstrap": (_st, [_vp, _vp, _vp, _vp, _u64, _vp]),
    "vsp_server_submit_keyset": (_st, [_vp, _vp, ctypes.POINTER(vsp_gate_desc), _u64, _u64, _vp, ctypes.POINTER(_u64)]),
    "vsp_mux": (_st, [_vp, _vp, _vp, _vp, _vp, _u64, _vp]),
    "vsp_autotune": (_st, [_vp, _u64, ctypes.c_char_p]),
    "vsp_tuning_get": (_st, [_vp, _u64, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "vsp_tuning_set_split": (_st, [_vp, _u64, _i32, ctypes.POINTER(ctypes.c_int)]),
    "vsp_tuning_set": (_st, [_vp, _u64, _i32, _i32]),
    "vsp_profile_enable": (_st, [_vp, _i32]),
    "vsp_profile_read": (_st, [_vp, _i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_u64)]),
    "vsp_measure_modp": (_st, [_i32, ctypes.c_uint32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "vsp_debug_external_product": (_st, [_vp, _vp, _vp, _vp, _u64, _vp]),
    "vsp_debug_polymul": (_st, [_vp, _vp, _vp, _vp, _u64, _vp]),
}


def lib() -> ctypes.CDLL:
    """The loaded libvsp (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name, None)
            if f is None:
                continue  # calling it raises AttributeError from the library object
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status: int, where: str) -> None:
    if status != VSP_OK:
        L = lib()
        raise VspError(status, where, f"{L.vsp_status_str(status).decode()}: {L.vsp_last_error().decode()}")


def _call(name, *args):
    check(getattr(lib(), name)(*args), name)


# ------------------------------------------------------------------ entry points
def vsp_context_create(bk_host, ksk_host, device: int = 0, params=DEFAULT_PARAMS) -> int:
    """bk_host / ksk_host: C-contiguous uint32 numpy arrays."""
    p = vsp_params(*params)
    out = _vp()
    _call("vsp_context_create", ctypes.byref(p), bk_host.ctypes.data, ksk_host.ctypes.data, device, ctypes.byref(out))
    return out.value


def vsp_context_destroy(ctx: int) -> None:
    _call("vsp_context_destroy", ctx)


def vsp_context_sync(ctx: int) -> None:
    _call("vsp_context_sync", ctx)


def vsp_gates(ctx, d_ops, d_in0, d_in1, d_out, B, mode=VSP_BATCHED, stream=None) -> None:
    _call("vsp_gates", ctx, d_ops, d_in0, d_in1, d_out, B, mode, stream)


def vsp_gates_noalloc(ctx, d_ops, d_in0, d_in1, d_out, B, mode=VSP_BATCHED, stream=None) -> None:
    _call("vsp_gates_noalloc", ctx, d_ops, d_in0, d_in1, d_out, B, mode, stream)


def vsp_gates_key_copies(ctx, d_ops, d_in0, d_in1, d_out, B, waves, copies, stream=None) -> float:
    """Blind-rotation milliseconds of a batch whose gate g reads key copy g mod copies."""
    ms = ctypes.c_double()
    _call("vsp_gates_key_copies", ctx, d_ops, d_in0, d_in1, d_out, B, waves, copies, stream, ctypes.byref(ms))
    return ms.value


def vsp_bootstrap_trlwe(ctx, d_ops, d_in0, d_in1, d_out, B, stream=None) -> None:
    _call("vsp_bootstrap_trlwe", ctx, d_ops, d_in0, d_in1, d_out, B, stream)


def gate_descs(gates) -> ctypes.Array:
    """(G, 3) integer array of (op, in0, in1) -> vsp_gate_desc[G]."""
    arr = (vsp_gate_desc * len(gates))()
    for i, (op, a, b) in enumerate(gates):
        arr[i].op, arr[i].in0, arr[i].in1 = int(op), int(a), int(b)
    return arr


def vsp_circuit_create(ctx, gates, ninputs: int) -> int:
    descs = gate_descs(gates)
    out = _vp()
    _call("vsp_circuit_create", ctx, descs, len(gates), ninputs, ctypes.byref(out))
    return out.value


def vsp_circuit_run(circ, d_inputs, d_wires, stream=None) -> None:
    _call("vsp_circuit_run", circ, d_inputs, d_wires, stream)


def vsp_circuit_run_timed(circ, d_inputs, d_wires, stream, nlevels: int):
    ms = (ctypes.c_float * nlevels)()
    _call("vsp_circuit_run_timed", circ, d_inputs, d_wires, stream, ms)
    return list(ms)


def vsp_circuit_info(circ):
    a, b = _u64(), _u64()
    _call("vsp_circuit_info", circ, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def vsp_circuit_destroy(circ) -> None:
    _call("vsp_circuit_destroy", circ)


def vsp_rom_read(ctx, d_rom, P, d_addr, v, w, d_out, R, stream=None) -> None:
    _call("vsp_rom_read", ctx, d_rom, P, d_addr, v, w, d_out, R, stream)


def vsp_ram_read(ctx, d_ram, v, w, d_addr, d_out, R, stream=None) -> None:
    _call("vsp_ram_read", ctx, d_ram, v, w, d_addr, d_out, R, stream)


def vsp_ram_write(ctx, d_ram, v, w, d_addr, d_flag, d_data, stream=None) -> None:
    _call("vsp_ram_write", ctx, d_ram, v, w, d_addr, d_flag, d_data, stream)


def vsp_server_create(ctx, mem_budget_bytes: int, max_batch: int) -> int:
    out = _vp()
    _call("vsp_server_create", ctx, mem_budget_bytes, max_batch, ctypes.byref(out))
    return out.value


def vsp_server_submit(srv, gates, ninputs: int, h_inputs) -> int:
    descs = gate_descs(gates)
    t = _u64()
    _call("vsp_server_submit", srv, descs, len(gates), ninputs, h_inputs.ctypes.data, ctypes.byref(t))
    return t.value


def vsp_machine_create(ctx, gates, ninputs: int, next_state) -> int:
    descs = gate_descs(gates)
    nxt = np.ascontiguousarray(next_state, dtype=np.uint32)
    out = _vp()
    _call("vsp_machine_create", ctx, descs, len(gates), ninputs, nxt.size, nxt.ctypes.data, ctypes.byref(out))
    return out.value


def vsp_machine_run(m, d_inputs, d_state, d_wires, ncycles: int, stream=None) -> None:
    _call("vsp_machine_run", m, d_inputs, d_state, d_wires, ncycles, stream)


def vsp_machine_destroy(m) -> None:
    _call("vsp_machine_destroy", m)


def vsp_keyset_create(ctx, bk_host, ksk_host) -> int:
    """bk_host / ksk_host: C-contiguous uint32 numpy arrays (another client's keys)."""
    out = _vp()
    _call("vsp_keyset_create", ctx, bk_host.ctypes.data, ksk_host.ctypes.data, ctypes.byref(out))
    return out.value


def vsp_keyset_destroy(k) -> None:
    _call("vsp_keyset_destroy", k)


def vsp_cbkey_create(ctx, bk2_host, pksk_host) -> int:
    """bk2_host: C-contiguous uint64 array [n][8][2][2048]; pksk_host: uint32 [2][2049][12][3][2][1024]."""
    out = _vp()
    _call("vsp_cbkey_create", ctx, bk2_host.ctypes.data, pksk_host.ctypes.data, ctypes.byref(out))
    return out.value


def vsp_machine_attach_ram(m, key, d_ram, v, w, addr_wires, flag_wire, data_wires, read_state) -> None:
    """addr_wires [v], data_wires [w], read_state [w]: sequences of ints (host)."""
    a = np.ascontiguousarray(addr_wires, dtype=np.uint32)
    d = np.ascontiguousarray(data_wires, dtype=np.uint32)
    r = np.ascontiguousarray(read_state, dtype=np.uint32)
    _call("vsp_machine_attach_ram", m, key, d_ram, v, w, a.ctypes.data, flag_wire, d.ctypes.data, r.ctypes.data)


def vsp_cbkey_destroy(k) -> None:
    _call("vsp_cbkey_destroy", k)


def vsp_cbkey_set_form(k, form: int) -> None:
    _call("vsp_cbkey_set_form", k, form)


def vsp_circuit_bootstrap(ctx, key, d_in, d_out, R, stream=None) -> None:
    _call("vsp_circuit_bootstrap", ctx, key, d_in, d_out, R, stream)


def vsp_server_submit_keyset(srv, keys, gates, ninputs: int, h_inputs) -> int:
    descs = gate_descs(gates)
    t = _u64()
    _call("vsp_server_submit_keyset", srv, keys, descs, len(gates), ninputs, h_inputs.ctypes.data, ctypes.byref(t))
    return t.value


def vsp_server_poll(srv, ticket: int, h_wires=None):
    done = _i32()
    lat = ctypes.c_double()
    _call("vsp_server_poll", srv, ticket, None if h_wires is None else h_wires.ctypes.data, ctypes.byref(done),
          ctypes.byref(lat))
    return bool(done.value), lat.value


def vsp_server_stats(srv):
    a, b, c = _u64(), _u64(), _u64()
    _call("vsp_server_stats", srv, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    return a.value, b.value, c.value


def vsp_server_destroy(srv) -> None:
    _call("vsp_server_destroy", srv)


def vsp_mux(ctx, d_sel, d_in1, d_in0, d_out, B, stream=None) -> None:
    _call("vsp_mux", ctx, d_sel, d_in1, d_in0, d_out, B, stream)


def vsp_autotune(ctx, max_batch: int, cache_path: str | None = None) -> None:
    _call("vsp_autotune", ctx, max_batch, cache_path.encode() if cache_path else None)


def vsp_tuning_get(ctx, B: int):
    """(blind-rotation waves per workgroup, key-switch tiled flag) used for a batch of B gates."""
    w = _i32()
    t = _i32()
    _call("vsp_tuning_get", ctx, B, ctypes.byref(w), ctypes.byref(t))
    return w.value, t.value


def vsp_tuning_set(ctx, B: int, br_waves: int, ks_form: int) -> None:
    _call("vsp_tuning_set", ctx, B, br_waves, ks_form)


def vsp_tuning_set_split(ctx, B: int, groups: int) -> int:
    """Pins the split form's workgroup count at the timed size covering B; returns the previous one."""
    prev = ctypes.c_int()
    _call("vsp_tuning_set_split", ctx, B, groups, ctypes.byref(prev))
    return prev.value


def vsp_profile_enable(ctx, on) -> None:
    """on: False/0 off, True/1 every launch, k > 1 every k-th launch of each kind."""
    _call("vsp_profile_enable", ctx, int(on))


def vsp_profile_read(ctx, which: int):
    """(total_ms, launches) of kernel class which: 0 blind rotation, 1 key switch, 2 prologue,
    3 step kernel of the matrix-core blind rotation."""
    ms = ctypes.c_double()
    cnt = _u64()
    _call("vsp_profile_read", ctx, which, ctypes.byref(ms), ctypes.byref(cnt))
    return ms.value, cnt.value


def vsp_measure_modp(device: int = 0, iters: int = 4096):
    """(general products mod p per second, lazy sums mod p per second) on the whole device."""
    mul, add = ctypes.c_double(), ctypes.c_double()
    _call("vsp_measure_modp", device, iters, ctypes.byref(mul), ctypes.byref(add))
    return mul.value, add.value


def vsp_debug_external_product(ctx, d_trgsw, d_x, d_out, J, stream=None) -> None:
    _call("vsp_debug_external_product", ctx, d_trgsw, d_x, d_out, J, stream)


def vsp_debug_polymul(ctx, d_a, d_b, d_out, J, stream=None) -> None:
    _call("vsp_debug_polymul", ctx, d_a, d_b, d_out, J, stream)
