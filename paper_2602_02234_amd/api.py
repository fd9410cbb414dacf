"""Python surface over the C ABI: a model handle, host and device evaluation,
and a ``torch.autograd.Function`` whose backward is the library's hand-written
backward pass.  PyTorch provides device memory and the stream only.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import DP_BF16, DP_FP32, check

_PREC = {"fp32": DP_FP32, "bf16": DP_BF16}


def _ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


def _box9(box):
    if box is None:
        return None
    b = np.asarray(box, dtype=np.float64)
    if b.shape == (3,):
        b = np.diag(b)
    return np.ascontiguousarray(b.reshape(3, 3))


class Model:
    """A model file loaded onto one GPU in one precision ("fp32" or "bf16")."""

    def __init__(self, path: str, precision: str = "fp32", device: int = 0):
        lib = _lib.load()
        h = C.c_void_p()
        check(lib.dp_model_load(path.encode(), _PREC[precision], device, C.byref(h)), "dp_model_load")
        self._h = h
        self.precision = precision
        self.device = device
        rc, sel, nt = C.c_double(), C.c_int(), C.c_int()
        check(lib.dp_model_info(h, C.byref(rc), C.byref(sel), C.byref(nt)), "dp_model_info")
        self.rc, self.sel, self.ntypes = rc.value, sel.value, nt.value
        self.last_status = 0
        # counts calls that replace the model's saved forward state; an autograd
        # backward compares it with the count its own forward left
        self.calls = 0

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().dp_model_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- host buffers
    def compute(self, coords, types, box=None, forces: bool = True, atom_energy: bool = False):
        """E (eV), F [N][3] (eV/A), virial [3][3] (eV) and optionally E_i, from host arrays."""
        self.calls += 1
        X = np.ascontiguousarray(coords, dtype=np.float64)
        T = np.ascontiguousarray(types, dtype=np.int32)
        n = X.shape[0]
        E = np.zeros(1)
        F = np.zeros((n, 3)) if forces else None
        V = np.zeros((3, 3)) if forces else None
        AE = np.zeros(n) if atom_energy else None
        b = _box9(box)
        st = _lib.load().dp_compute(self._h, n, _ptr(X), _ptr(T), _ptr(b), _ptr(E), _ptr(F), _ptr(V), _ptr(AE))
        self.last_status = check(st, "dp_compute")
        out = {"E": float(E[0])}
        if forces:
            out["F"], out["virial"] = F, V
        if atom_energy:
            out["E_i"] = AE
        return out

    def neighbors(self, coords, box=None):
        self.calls += 1
        X = np.ascontiguousarray(coords, dtype=np.float64)
        n = X.shape[0]
        nl = np.zeros((n, self.sel), dtype=np.int32)
        nn = np.zeros(n, dtype=np.int32)
        ov = C.c_int64()
        b = _box9(box)
        st = _lib.load().dp_debug_neighbors(self._h, n, _ptr(X), _ptr(b), _ptr(nl), _ptr(nn), C.byref(ov))
        self.last_status = check(st, "dp_debug_neighbors")
        return nl, nn, int(ov.value)

    def pair_grads(self, natoms: int):
        """g[i][s] = dE_i/dDelta_ij of the last backward pass, [natoms][sel][3]."""
        g = np.zeros((natoms, self.sel, 4), dtype=np.float32)
        check(_lib.load().dp_debug_pair_grads(self._h, natoms, _ptr(g)), "dp_debug_pair_grads")
        return g[:, :, :3]

    # ---------------------------------------------------------------- step options
    def set_skin(self, skin: float, rebuild_every: int = 10):
        """Reuse neighbour lists built within rc + skin for up to rebuild_every calls (0 = off)."""
        check(_lib.load().dp_set_skin(self._h, float(skin), int(rebuild_every)), "dp_set_skin")

    def skin_stats(self):
        b, f = np.zeros(1, dtype=np.int64), np.zeros(1, dtype=np.int64)
        check(_lib.load().dp_skin_stats(self._h, _ptr(b), _ptr(f)), "dp_skin_stats")
        return {"builds": int(b[0]), "forced": int(f[0])}

    @property
    def nheads(self) -> int:
        k = C.c_int()
        check(_lib.load().dp_model_heads(self._h, C.byref(k)), "dp_model_heads")
        return k.value

    def set_head_weights(self, weights):
        """E = sum_h w_h E^h of the fitting heads (forces and virial follow)."""
        w = np.ascontiguousarray(weights, dtype=np.float64)
        check(_lib.load().dp_set_head_weights(self._h, len(w), _ptr(w)), "dp_set_head_weights")

    def head_energies(self, nsys: int = 1):
        """Each head's energy E^h of the last step, [nsys][nheads]."""
        out = np.zeros((nsys, self.nheads))
        check(_lib.load().dp_head_energies(self._h, nsys, _ptr(out)), "dp_head_energies")
        return out

    def set_chunk(self, chunk_atoms: int):
        """Evaluate the centres of larger systems in chunks of chunk_atoms (0 = off)."""
        check(_lib.load().dp_set_chunk(self._h, int(chunk_atoms)), "dp_set_chunk")

    def set_graph(self, enable: bool = True):
        """Capture each step configuration in a HIP graph and replay it."""
        check(_lib.load().dp_set_graph(self._h, 1 if enable else 0), "dp_set_graph")

    # ---------------------------------------------------------------- timing
    PHASES = ("neighbors", "descriptor_fwd", "fitting", "energy_reduce", "descriptor_bwd", "forces_virial")

    def profile(self, enable: bool = True):
        check(_lib.load().dp_profile_enable(self._h, 1 if enable else 0), "dp_profile_enable")

    def profile_read(self):
        """{phase: (total ms, calls)} accumulated since profile(True)."""
        ms = np.zeros(8)
        calls = np.zeros(8, dtype=np.int64)
        k = _lib.load().dp_profile_read(self._h, _ptr(ms), _ptr(calls), 8)
        return {self.PHASES[i]: (float(ms[i]), int(calls[i])) for i in range(min(k, len(self.PHASES)))}

    # ---------------------------------------------------------------- device buffers
    def compute_device(self, coords, types, box=None, forces=None, virial=None, energy=None, atom_energy=None,
                       stream=None):
        """Evaluate on torch CUDA tensors (float64 coords [N][3], int32 types [N]); outputs are written in place.

        Returns the energy tensor [1].  ``forces``/``virial`` None (both) runs the energy pass only.
        """
        self.calls += 1
        import torch
        n = coords.shape[0]
        assert coords.is_cuda and coords.dtype == torch.float64 and coords.is_contiguous()
        assert types.is_cuda and types.dtype == torch.int32 and types.is_contiguous()
        if energy is None:
            energy = torch.empty(1, dtype=torch.float64, device=coords.device)
        s = stream if stream is not None else torch.cuda.current_stream(coords.device).cuda_stream
        b = _box9(box)

        def dp(t):
            return C.c_void_p(t.data_ptr()) if t is not None else None

        st = _lib.load().dp_compute_device(self._h, n, dp(coords), dp(types), _ptr(b), dp(energy), dp(forces),
                                           dp(virial), dp(atom_energy), C.c_void_p(s))
        self.last_status = check(st, "dp_compute_device")
        return energy

    def compute_owned_device(self, coords, types, n_owned: int, box=None, forces=None, virial=None, energy=None,
                             atom_energy=None, stream=None):
        """One share of a decomposed system (dp_compute_owned_device): the first n_owned atoms
        are owned, the rest ghosts.  Torch CUDA tensors; outputs written in place."""
        self.calls += 1
        import torch
        n = coords.shape[0]
        assert coords.is_cuda and coords.dtype == torch.float64 and coords.is_contiguous()
        assert types.is_cuda and types.dtype == torch.int32 and types.is_contiguous()
        if energy is None:
            energy = torch.empty(1, dtype=torch.float64, device=coords.device)
        s = stream if stream is not None else torch.cuda.current_stream(coords.device).cuda_stream
        b = _box9(box)

        def dp(t):
            return C.c_void_p(t.data_ptr()) if t is not None else None

        st = _lib.load().dp_compute_owned_device(self._h, n, int(n_owned), dp(coords), dp(types), _ptr(b), dp(energy),
                                                 dp(forces), dp(virial), dp(atom_energy), C.c_void_p(s))
        self.last_status = check(st, "dp_compute_owned_device")
        return energy

    def compute_batch(self, systems, forces: bool = True):
        """Several periodic systems [(coords, types, box), ...] in one batched step (through
        device buffers).  Returns one dict per system (E, F, virial)."""
        self.calls += 1
        import torch
        dev = torch.device("cuda", self.device)
        ns = np.array([len(t) for _, t, _ in systems], dtype=np.int64)
        X = torch.tensor(np.concatenate([np.asarray(c, dtype=np.float64) for c, _, _ in systems]), device=dev)
        T = torch.tensor(np.concatenate([np.asarray(t, dtype=np.int32) for _, t, _ in systems]), device=dev)
        boxes = np.ascontiguousarray(np.stack([_box9(b) for _, _, b in systems]))
        k = len(systems)
        E = torch.zeros(k, dtype=torch.float64, device=dev)
        F = torch.zeros((int(ns.sum()), 3), dtype=torch.float64, device=dev) if forces else None
        V = torch.zeros((k, 9), dtype=torch.float64, device=dev) if forces else None

        def dp(t):
            return C.c_void_p(t.data_ptr()) if t is not None else None

        s = torch.cuda.current_stream(dev).cuda_stream
        st = _lib.load().dp_compute_batch_device(self._h, k, _ptr(ns), _ptr(boxes), dp(X), dp(T), dp(E), dp(F),
                                                 dp(V), C.c_void_p(s))
        self.last_status = check(st, "dp_compute_batch_device")
        out, off = [], 0
        Eh = E.cpu().numpy()
        Fh = F.cpu().numpy() if forces else None
        Vh = V.cpu().numpy() if forces else None
        for q in range(k):
            d = {"E": float(Eh[q])}
            if forces:
                d["F"] = Fh[off:off + ns[q]]
                d["virial"] = Vh[q].reshape(3, 3)
            off += ns[q]
            out.append(d)
        return out

    def nve(self, coords, velocities, types, masses, box, dt_fs: float, steps: int):
        """Velocity-Verlet NVE on the device (torch float64 coords/velocities advanced in place).
        Returns (epot, ekin), arrays of steps + 1 energies in eV."""
        self.calls += 1
        import torch
        assert coords.is_cuda and coords.dtype == torch.float64 and coords.is_contiguous()
        assert velocities.is_cuda and velocities.dtype == torch.float64 and velocities.is_contiguous()
        assert types.is_cuda and types.dtype == torch.int32
        m = np.ascontiguousarray(masses, dtype=np.float64)
        ep, ek = np.zeros(steps + 1), np.zeros(steps + 1)
        s = torch.cuda.current_stream(coords.device).cuda_stream
        st = _lib.load().dp_nve_run(self._h, coords.shape[0], C.c_void_p(coords.data_ptr()),
                                    C.c_void_p(velocities.data_ptr()), C.c_void_p(types.data_ptr()), _ptr(m),
                                    _ptr(_box9(box)), float(dt_fs), int(steps), _ptr(ep), _ptr(ek), C.c_void_p(s))
        self.last_status = check(st, "dp_nve_run")
        return ep, ek

    def backward_device(self, grad_energy, grad_coords, virial=None, stream=None):
        self.calls += 1
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(grad_coords.device).cuda_stream
        st = _lib.load().dp_backward_device(self._h, C.c_void_p(grad_energy.data_ptr()),
                                            C.c_void_p(grad_coords.data_ptr()),
                                            C.c_void_p(virial.data_ptr()) if virial is not None else None,
                                            C.c_void_p(s))
        check(st, "dp_backward_device")


class Server:
    """Continuous-batching server (dp_server_*): submit host systems, wait for results."""

    def __init__(self, model: Model, hbm_budget_bytes: int, max_inflight: int = 3):
        lib = _lib.load()
        h = C.c_void_p()
        check(lib.dp_server_create(model._h, int(hbm_budget_bytes), int(max_inflight), C.byref(h)),
              "dp_server_create")
        self._h = h
        self.model = model
        self._n = {}

    def footprint(self, natoms: int) -> int:
        return int(_lib.load().dp_server_footprint(self.model._h, int(natoms)))

    def submit(self, coords, types, box) -> int:
        X = np.ascontiguousarray(coords, dtype=np.float64)
        T = np.ascontiguousarray(types, dtype=np.int32)
        b = _box9(box)
        rid = C.c_uint64()
        check(_lib.load().dp_submit(self._h, X.shape[0], _ptr(X), _ptr(T), _ptr(b), C.byref(rid)), "dp_submit")
        self._n[rid.value] = X.shape[0]
        return rid.value

    def wait(self, rid: int, timeout: float = -1.0):
        n = self._n[rid]
        E, F, V, lat = np.zeros(1), np.zeros((n, 3)), np.zeros((3, 3)), np.zeros(1)
        st = _lib.load().dp_wait(self._h, C.c_uint64(rid), float(timeout), _ptr(E), _ptr(F), _ptr(V), _ptr(lat))
        if st != -10:
            self._n.pop(rid, None)
        check(st, "dp_wait")
        return {"E": float(E[0]), "F": F, "virial": V, "latency": float(lat[0]), "status": st}

    def stats(self):
        p50, p99, rate = np.zeros(1), np.zeros(1), np.zeros(1)
        done, nb, mb = np.zeros(1, dtype=np.int64), np.zeros(1, dtype=np.int64), np.zeros(1, dtype=np.int64)
        check(_lib.load().dp_server_stats(self._h, _ptr(p50), _ptr(p99), _ptr(rate), _ptr(done), _ptr(nb), _ptr(mb)),
              "dp_server_stats")
        return {"p50_s": float(p50[0]), "p99_s": float(p99[0]), "atom_evals_per_s": float(rate[0]),
                "completed": int(done[0]), "batches": int(nb[0]), "max_batch_atoms": int(mb[0])}

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().dp_server_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GnnModel:
    """A GNN-variant model file (message passing over edges and angles) on one GPU,
    in one precision ("fp32" or "bf16")."""

    def __init__(self, path: str, precision: str = "fp32", device: int = 0):
        lib = _lib.load()
        h = C.c_void_p()
        check(lib.dp_gnn_load(path.encode(), _PREC[precision], device, C.byref(h)), "dp_gnn_load")
        self._h = h
        self.precision = precision
        self.device = device
        rc, rca, sel, asel = C.c_double(), C.c_double(), C.c_int(), C.c_int()
        check(lib.dp_gnn_info(h, C.byref(rc), C.byref(rca), C.byref(sel), C.byref(asel)), "dp_gnn_info")
        self.rc, self.rca, self.sel, self.asel = rc.value, rca.value, sel.value, asel.value
        self.last_status = 0

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().dp_gnn_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def compute_device(self, coords, types, box=None, forces=None, virial=None, energy=None, atom_energy=None,
                       stream=None):
        """Evaluate on torch CUDA tensors (float64 coords [N][3], int32 types [N]); outputs written in place."""
        import torch
        n = coords.shape[0]
        assert coords.is_cuda and coords.dtype == torch.float64 and coords.is_contiguous()
        assert types.is_cuda and types.dtype == torch.int32 and types.is_contiguous()
        if energy is None:
            energy = torch.empty(1, dtype=torch.float64, device=coords.device)
        s = stream if stream is not None else torch.cuda.current_stream(coords.device).cuda_stream
        b = _box9(box)

        def dp(t):
            return C.c_void_p(t.data_ptr()) if t is not None else None

        st = _lib.load().dp_gnn_compute_device(self._h, n, dp(coords), dp(types), _ptr(b), dp(energy), dp(forces),
                                               dp(virial), dp(atom_energy), C.c_void_p(s))
        self.last_status = check(st, "dp_gnn_compute_device")
        return energy

    def compute(self, coords, types, box=None, forces: bool = True, atom_energy: bool = False):
        """E, F, virial (and E_i) from host arrays, through device copies made with torch."""
        import torch
        dev = torch.device("cuda", self.device)
        X = torch.tensor(np.ascontiguousarray(coords, dtype=np.float64), device=dev)
        T = torch.tensor(np.ascontiguousarray(types, dtype=np.int32), device=dev)
        n = X.shape[0]
        F = torch.zeros((n, 3), dtype=torch.float64, device=dev) if forces else None
        V = torch.zeros(9, dtype=torch.float64, device=dev) if forces else None
        AE = torch.zeros(n, dtype=torch.float64, device=dev) if atom_energy else None
        E = self.compute_device(X, T, box, forces=F, virial=V, atom_energy=AE)
        torch.cuda.synchronize(dev)
        out = {"E": float(E.item())}
        if forces:
            out["F"], out["virial"] = F.cpu().numpy(), V.cpu().numpy().reshape(3, 3)
        if atom_energy:
            out["E_i"] = AE.cpu().numpy()
        return out

    def angles(self) -> int:
        """Angles of the last successful step."""
        return self.graph_size()[2]

    def graph_size(self):
        """(edges, angle-list edges, angles) of the last successful step."""
        e, c, a = C.c_int64(), C.c_int64(), C.c_int64()
        check(_lib.load().dp_gnn_graph_size(self._h, C.byref(e), C.byref(c), C.byref(a)), "dp_gnn_graph_size")
        return int(e.value), int(c.value), int(a.value)

    PHASES = ("lists", "layers_fwd", "layers_bwd", "forces")

    def profile(self, enable: bool = True):
        check(_lib.load().dp_gnn_profile_enable(self._h, 1 if enable else 0), "dp_gnn_profile_enable")

    def profile_read(self):
        """{phase: (total ms, calls)} accumulated since profile(True)."""
        ms = np.zeros(4)
        calls = np.zeros(4, dtype=np.int64)
        k = _lib.load().dp_gnn_profile_read(self._h, _ptr(ms), _ptr(calls), 4)
        return {self.PHASES[i]: (float(ms[i]), int(calls[i])) for i in range(k)}


class RepModel:
    """A repformer-style model file (pair and node features, gated self-attention over
    the neighbours' pair features, neighbour-to-neighbour message passing) on one GPU,
    float32."""

    PHASES = ("lists", "layers_fwd", "layers_bwd", "forces")

    def __init__(self, path: str, device: int = 0):
        lib = _lib.load()
        h = C.c_void_p()
        check(lib.dp_rep_load(path.encode(), device, C.byref(h)), "dp_rep_load")
        self._h = h
        self.device = device
        self.last_status = 0

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().dp_rep_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def compute_device(self, coords, types, box=None, forces=None, virial=None, energy=None, atom_energy=None,
                       stream=None):
        """Evaluate on torch CUDA tensors (float64 coords [N][3], int32 types [N]); outputs written in place."""
        import torch
        n = coords.shape[0]
        assert coords.is_cuda and coords.dtype == torch.float64 and coords.is_contiguous()
        assert types.is_cuda and types.dtype == torch.int32 and types.is_contiguous()
        if energy is None:
            energy = torch.empty(1, dtype=torch.float64, device=coords.device)
        s = stream if stream is not None else torch.cuda.current_stream(coords.device).cuda_stream
        b = _box9(box)

        def dp(t):
            return C.c_void_p(t.data_ptr()) if t is not None else None

        st = _lib.load().dp_rep_compute_device(self._h, n, dp(coords), dp(types), _ptr(b), dp(energy), dp(forces),
                                               dp(virial), dp(atom_energy), C.c_void_p(s))
        self.last_status = check(st, "dp_rep_compute_device")
        return energy

    def compute(self, coords, types, box=None, forces: bool = True, atom_energy: bool = False):
        """E, F, virial (and E_i) from host arrays, through device copies made with torch."""
        import torch
        dev = torch.device("cuda", self.device)
        X = torch.tensor(np.ascontiguousarray(coords, dtype=np.float64), device=dev)
        T = torch.tensor(np.ascontiguousarray(types, dtype=np.int32), device=dev)
        n = X.shape[0]
        F = torch.zeros((n, 3), dtype=torch.float64, device=dev) if forces else None
        V = torch.zeros(9, dtype=torch.float64, device=dev) if forces else None
        AE = torch.zeros(n, dtype=torch.float64, device=dev) if atom_energy else None
        E = self.compute_device(X, T, box, forces=F, virial=V, atom_energy=AE)
        torch.cuda.synchronize(dev)
        out = {"E": float(E.item())}
        if forces:
            out["F"], out["virial"] = F.cpu().numpy(), V.cpu().numpy().reshape(3, 3)
        if atom_energy:
            out["E_i"] = AE.cpu().numpy()
        return out

    def edges(self) -> int:
        v = C.c_int64()
        check(_lib.load().dp_rep_edges(self._h, C.byref(v)), "dp_rep_edges")
        return int(v.value)

    def profile(self, enable: bool = True):
        check(_lib.load().dp_rep_profile_enable(self._h, 1 if enable else 0), "dp_rep_profile_enable")

    def profile_read(self):
        ms = np.zeros(4)
        calls = np.zeros(4, dtype=np.int64)
        k = _lib.load().dp_rep_profile_read(self._h, _ptr(ms), _ptr(calls), 4)
        return {self.PHASES[i]: (float(ms[i]), int(calls[i])) for i in range(k)}


def _autograd_function():
    import torch

    class DPEnergy(torch.autograd.Function):
        """E = DPEnergy.apply(coords, types, model, box); dE/dcoords from the library's backward kernels."""

        @staticmethod
        def forward(ctx, coords, types, model, box):
            x = coords.detach().contiguous()
            t = types.contiguous()
            E = model.compute_device(x, t, box)
            ctx.model = model
            ctx.box = box
            ctx.token = model.calls
            ctx.save_for_backward(x, t)
            return E.reshape(())

        @staticmethod
        def backward(ctx, gE):
            x, types = ctx.saved_tensors
            model = ctx.model
            if model.calls != ctx.token:
                # another call ran on the model since this forward: its saved state is
                # not this graph's, so the energy pass is redone at this forward's inputs
                model.compute_device(x, types, ctx.box)
            g = torch.empty(x.shape, dtype=torch.float64, device=x.device)
            gE = gE.detach().reshape(1).to(torch.float64).contiguous()
            model.backward_device(gE, g)
            return g, None, None, None

    return DPEnergy


_DPEnergy = None


def energy(model: Model, coords, types, box=None):
    """Differentiable total energy of torch CUDA coordinates: forces = -autograd.grad(E, coords)."""
    global _DPEnergy
    if _DPEnergy is None:
        _DPEnergy = _autograd_function()
    return _DPEnergy.apply(coords, types, model, box)
