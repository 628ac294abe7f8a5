"""ctypes binding of libgridff (include/gridff.h): argument marshalling only.

Every step of the path runs in the library's HIP kernels; torch is used for device
memory and streams.  The functions keep the C names without the ``gff_`` prefix.
Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgridff.so")

STORE_F32, STORE_F16, STORE_TRILINEAR = 0, 1, 2
MODE_FIRE, MODE_NVE, MODE_LANGEVIN = 0, 1, 2
K_B = 8.617333262e-5                    # Boltzmann constant [eV/K]
REP_CONVERGED, REP_OUT_OF_DOMAIN, REP_NONFINITE, REP_MAXSTEPS = 1, 2, 4, 8


class GffError(RuntimeError):
    pass


class Substrate(C.Structure):
    _fields_ = [("n_atoms", C.c_int), ("pos_h", C.c_void_p), ("q_h", C.c_void_p), ("eps_h", C.c_void_p),
                ("R_h", C.c_void_p), ("Lx", C.c_double), ("Ly", C.c_double)]


class GridSpec(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("x0", C.c_double), ("y0", C.c_double),
                ("z0", C.c_double), ("dz", C.c_double), ("alpha", C.c_double), ("rcut", C.c_double),
                ("k_e", C.c_double)]


class Grid(C.Structure):
    _fields_ = [("storage", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("x0", C.c_float), ("y0", C.c_float), ("z0", C.c_float),
                ("dx", C.c_float), ("dy", C.c_float), ("dz", C.c_float),
                ("d_coef", C.c_void_p), ("d_scale", C.c_void_p)]


class MolType(C.Structure):
    _fields_ = [("n_atoms", C.c_int), ("eps", C.c_void_p), ("R", C.c_void_p), ("q", C.c_void_p),
                ("mass", C.c_void_p),
                ("n_bonds", C.c_int), ("bonds", C.c_void_p), ("bond_k", C.c_void_p), ("bond_r0", C.c_void_p),
                ("n_angles", C.c_int), ("angles", C.c_void_p), ("angle_k", C.c_void_p), ("angle_cos0", C.c_void_p),
                ("n_tors", C.c_int), ("tors", C.c_void_p), ("tors_V", C.c_void_p), ("tors_n", C.c_void_p),
                ("tors_phi0", C.c_void_p),
                ("n_rot", C.c_int), ("rot_quads", C.c_void_p), ("rot_mask", C.c_void_p),
                ("ref_pos", C.c_void_p)]


class Launch(C.Structure):
    _fields_ = [("block_threads", C.c_int), ("reps_per_block", C.c_int), ("grid_blocks", C.c_int),
                ("lanes_per_atom", C.c_int)]


class RelaxParams(C.Structure):
    _fields_ = [("mode", C.c_int), ("n_steps", C.c_int), ("include_intra", C.c_int), ("dt", C.c_float),
                ("f_conv", C.c_float), ("max_disp", C.c_float), ("fire_finc", C.c_float),
                ("fire_fdec", C.c_float), ("fire_alpha0", C.c_float), ("fire_falpha", C.c_float),
                ("fire_dtmax", C.c_float), ("fire_nmin", C.c_int), ("drift_every", C.c_int),
                ("kT", C.c_float), ("gamma", C.c_float), ("seed", C.c_ulonglong), ("round", C.c_uint),
                ("check_every", C.c_int)]


class State(C.Structure):
    _fields_ = [("d_pos", C.c_void_p), ("d_vel", C.c_void_p), ("d_fire_dt", C.c_void_p),
                ("d_fire_alpha", C.c_void_p), ("d_fire_npos", C.c_void_p), ("d_status", C.c_void_p),
                ("d_fixed_atom", C.c_void_p), ("d_fixed_pos", C.c_void_p)]


EXPORTS = [
    "gff_status_string", "gff_build_grid_workspace_bytes", "gff_build_grid", "gff_fit_workspace_bytes",
    "gff_fit_bspline", "gff_grid_bytes", "gff_pack_grid", "gff_topology_create", "gff_topology_destroy",
    "gff_plan_create", "gff_plan_destroy", "gff_plan_n_atoms", "gff_plan_n_packs", "gff_plan_atom_offsets",
    "gff_eval_forces", "gff_interp_points", "gff_relax_batch", "gff_relax_occupancy",
]

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise GffError(f"{LIB_PATH} is missing: build it with paper_2508_15522_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        L.gff_status_string.restype = C.c_char_p
        for n in ("gff_build_grid_workspace_bytes", "gff_fit_workspace_bytes", "gff_grid_bytes",
                  "gff_dedupe_rmsd_workspace_bytes"):
            getattr(L, n).restype = C.c_size_t
        for n in ("gff_build_grid", "gff_fit_bspline", "gff_pack_grid", "gff_topology_create", "gff_plan_create",
                  "gff_plan_atom_offsets", "gff_eval_forces", "gff_interp_points", "gff_relax_batch",
                  "gff_plan_n_atoms", "gff_plan_n_packs"):
            getattr(L, n).restype = C.c_int
        _lib = L
    return _lib


def check(rc):
    if rc != 0:
        raise GffError(f"libgridff: {lib().gff_status_string(rc).decode()} ({rc})")


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------------ grid build / fit / pack
class _Keep:
    def __init__(self):
        self.arrays = []

    def np(self, a, dtype):
        a = np.ascontiguousarray(a, dtype=dtype)
        self.arrays.append(a)
        return a.ctypes.data_as(C.c_void_p)


def grid_spec(nx, ny, nz, x0, y0, z0, dz, alpha=1.6, rcut=17.0, k_e=0.0):
    return GridSpec(nx, ny, nz, x0, y0, z0, dz, alpha, rcut, k_e)


def substrate(sub, keep):
    return Substrate(sub.n, keep.np(sub.pos, np.float64), keep.np(sub.q, np.float64),
                     keep.np(sub.eps, np.float64), keep.np(sub.R, np.float64), sub.Lx, sub.Ly)


def build_grid_workspace_bytes(spec, sub):
    keep = _Keep()
    s = substrate(sub, keep)
    return lib().gff_build_grid_workspace_bytes(C.byref(spec), C.byref(s))


def build_grid(sub, spec, d_V, d_work, stream=None):
    keep = _Keep()
    s = substrate(sub, keep)
    check(lib().gff_build_grid(C.byref(s), C.byref(spec), _ptr(d_V), _ptr(d_work),
                               C.c_size_t(d_work.numel() * d_work.element_size()), _stream(stream)))


def fit_workspace_bytes(spec):
    return lib().gff_fit_workspace_bytes(C.byref(spec))


def fit_bspline(spec, d_V, d_B, d_work, stream=None):
    check(lib().gff_fit_bspline(C.byref(spec), _ptr(d_V), _ptr(d_B), _ptr(d_work),
                                C.c_size_t(d_work.numel() * d_work.element_size()), _stream(stream)))


def grid_bytes(spec, storage):
    return lib().gff_grid_bytes(C.byref(spec), C.c_int(storage))


def pack_grid(spec, d_B, storage, d_coef, d_scale, stream=None):
    check(lib().gff_pack_grid(C.byref(spec), _ptr(d_B), C.c_int(storage), _ptr(d_coef), _ptr(d_scale),
                              _stream(stream)))


def grid(spec, storage, d_coef, d_scale, Lx, Ly):
    """gff_grid descriptor for a packed grid of `spec` (lateral spacing Lx/nx, Ly/ny)."""
    return Grid(storage, spec.nx, spec.ny, spec.nz, spec.x0, spec.y0, spec.z0, Lx / spec.nx, Ly / spec.ny,
                spec.dz, d_coef.data_ptr(), None if d_scale is None else d_scale.data_ptr())


# ------------------------------------------------------------------ topology / plan
class Topology:
    def __init__(self, mols, alpha=1.6, k_e=0.0):
        self.keep = _Keep()
        arr = (MolType * len(mols))()
        for t, m in enumerate(mols):
            k = self.keep
            nrot = len(m.rot_quads)
            arr[t] = MolType(
                m.n, k.np(m.eps, np.float32), k.np(m.R, np.float32), k.np(m.q, np.float32), k.np(m.mass, np.float32),
                len(m.bonds), k.np(m.bonds.reshape(-1, 2), np.int32), k.np(m.bond_k, np.float32),
                k.np(m.bond_r0, np.float32),
                len(m.angles), k.np(m.angles.reshape(-1, 3), np.int32), k.np(m.angle_k, np.float32),
                k.np(m.angle_cos0, np.float32),
                len(m.tors), k.np(m.tors.reshape(-1, 4), np.int32), k.np(m.tors_V, np.float32),
                k.np(m.tors_n, np.int32), k.np(m.tors_phi0, np.float32),
                nrot, k.np(m.rot_quads.reshape(-1, 4) if nrot else np.zeros((1, 4)), np.int32),
                k.np(m.rot_masks.reshape(nrot, m.n) if nrot else np.zeros((1, m.n)), np.uint8),
                k.np(m.pos, np.float32))
        self.handle = C.c_void_p()
        check(lib().gff_topology_create(arr, C.c_int(len(mols)), C.c_float(alpha), C.c_float(k_e),
                                        C.byref(self.handle)))
        self.mols = mols

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.gff_topology_destroy(self.handle)
            self.handle = None


class Plan:
    def __init__(self, topo: Topology, rep_type, block_threads=256, reps_per_block=0, grid_blocks=0,
                 lanes_per_atom=1):
        rt = np.ascontiguousarray(rep_type, dtype=np.int32)
        self.n_rep = len(rt)
        self.handle = C.c_void_p()
        self.launch = Launch(block_threads, reps_per_block, grid_blocks, lanes_per_atom)
        check(lib().gff_plan_create(topo.handle, C.c_int(self.n_rep), rt.ctypes.data_as(C.c_void_p),
                                    C.byref(self.launch), C.byref(self.handle)))
        self.n_atoms = lib().gff_plan_n_atoms(self.handle)
        self.n_packs = lib().gff_plan_n_packs(self.handle)
        off = np.zeros(self.n_rep + 1, np.int32)
        check(lib().gff_plan_atom_offsets(self.handle, off.ctypes.data_as(C.c_void_p)))
        self.atom_off = off
        self.rep_type = rt

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.gff_plan_destroy(self.handle)
            self.handle = None


def relax_occupancy(grid_desc, plan, mode):
    """(resident blocks per compute unit, dynamic LDS bytes per block) of the replica kernel
    for this grid and plan; mode MODE_FIRE, MODE_NVE or -1 (single evaluation)."""
    blocks = C.c_int(0)
    lds = C.c_size_t(0)
    check(lib().gff_relax_occupancy(C.byref(grid_desc), plan.handle, C.c_int(mode), C.byref(blocks), C.byref(lds)))
    return blocks.value, lds.value


# ------------------------------------------------------------------ evaluation / relaxation
def eval_forces(grid_desc, topo, plan, include_intra, d_pos, d_F, d_E_atom=None, d_E_rep=None, d_status=None,
                stream=None):
    check(lib().gff_eval_forces(C.byref(grid_desc), topo.handle, plan.handle, C.c_int(int(include_intra)),
                                _ptr(d_pos), _ptr(d_F), _ptr(d_E_atom), _ptr(d_E_rep), _ptr(d_status),
                                _stream(stream)))


def interp_points(grid_desc, d_pos, d_plq, d_F, d_E=None, stream=None):
    n = d_pos.shape[-1]
    check(lib().gff_interp_points(C.byref(grid_desc), C.c_int(n), _ptr(d_pos), _ptr(d_plq), _ptr(d_F), _ptr(d_E),
                                  _stream(stream)))


def relax_params(mode=MODE_FIRE, n_steps=1000, include_intra=True, dt=0.5, f_conv=1e-4, max_disp=0.1,
                 finc=1.1, fdec=0.5, alpha0=0.1, falpha=0.99, dtmax=0.1, nmin=5, drift_every=1,
                 T=300.0, gamma=0.01, seed=0, rnd=0, check_every=1):
    """T is the Langevin bath temperature in K (kT = k_B T in the C struct)."""
    return RelaxParams(mode, n_steps, int(include_intra), dt, f_conv, max_disp, finc, fdec, alpha0, falpha,
                       dtmax, nmin, drift_every, K_B * T, gamma, seed, rnd, check_every)


def _state(st):
    g = lambda k: st[k].data_ptr() if k in st and st[k] is not None else None
    return State(g("pos"), g("vel"), g("fire_dt"), g("fire_alpha"), g("fire_npos"), g("status"), g("fixed_atom"),
                 g("fixed_pos"))


def relax_batch(grid_desc, topo, plan, params, st, d_E_rep, d_fnorm, d_steps, d_drift=None, stream=None):
    """st: dict of torch tensors pos, vel, fire_dt, fire_alpha, fire_npos, status and, for a
    restraint, fixed_atom (int32 [n_rep]) and fixed_pos (float32 [n_rep][3])."""
    state = _state(st)
    check(lib().gff_relax_batch(C.byref(grid_desc), topo.handle, plan.handle, C.byref(params), C.byref(state),
                                _ptr(d_E_rep), _ptr(d_fnorm), _ptr(d_steps), _ptr(d_drift), _stream(stream)))


EXPORTS += ["gff_relax_scan"]


def relax_scan(grid_desc, topo, plan, params, st, d_path, n_points, moves_per_point, dt0, d_E_points,
               d_steps_points=None, d_status_points=None, d_pos_points=None, d_E_rep=None, d_fnorm=None, d_steps=None,
               stream=None):
    """A whole restrained scan in one FIRE launch; st as for relax_batch with fixed_atom."""
    check(lib().gff_relax_scan(C.byref(grid_desc), topo.handle, plan.handle, C.byref(params), C.byref(_state(st)),
                               _ptr(d_path), C.c_int(n_points), C.c_int(moves_per_point), C.c_float(dt0),
                               _ptr(d_E_points), _ptr(d_steps_points), _ptr(d_status_points), _ptr(d_pos_points),
                               _ptr(d_E_rep), _ptr(d_fnorm), _ptr(d_steps), _stream(stream)))


# ------------------------------------------------------------------ all-atom comparison mode
EXPORTS += ["gff_direct_create", "gff_direct_destroy", "gff_eval_forces_direct", "gff_relax_batch_direct"]


class Direct:
    """Substrate atoms on the device for the all-atom comparison (cell + lateral images
    |a|, |b| <= n_img, bare sums, no cutoff)."""

    def __init__(self, sub, alpha=1.6, n_img=1):
        keep = _Keep()
        s = substrate(sub, keep)
        self.handle = C.c_void_p()
        check(lib().gff_direct_create(C.byref(s), C.c_float(alpha), C.c_int(n_img), C.byref(self.handle)))
        self.n_img = n_img

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.gff_direct_destroy(self.handle)
            self.handle = None


def eval_forces_direct(direct, topo, plan, include_intra, d_pos, d_F, d_E_atom=None, d_E_rep=None, d_status=None,
                       stream=None):
    check(lib().gff_eval_forces_direct(direct.handle, topo.handle, plan.handle, C.c_int(int(include_intra)),
                                       _ptr(d_pos), _ptr(d_F), _ptr(d_E_atom), _ptr(d_E_rep), _ptr(d_status),
                                       _stream(stream)))


def relax_batch_direct(direct, topo, plan, params, st, d_E_rep, d_fnorm, d_steps, d_drift=None, stream=None):
    state = _state(st)
    check(lib().gff_relax_batch_direct(direct.handle, topo.handle, plan.handle, C.byref(params), C.byref(state),
                                       _ptr(d_E_rep), _ptr(d_fnorm), _ptr(d_steps), _ptr(d_drift),
                                       _stream(stream)))


# ------------------------------------------------------------------ proposals / minima
EXPORTS += ["gff_propose_uniform", "gff_pose_from_dof", "gff_encode_pose", "gff_decode_dof", "gff_dedupe_energy",
            "gff_mlp_n_params", "gff_mlp_create", "gff_mlp_destroy", "gff_mlp_get_params", "gff_mlp_workspace_bytes",
            "gff_mlp_forward", "gff_mlp_train_step", "gff_imle_select", "gff_normal_philox", "gff_gemm_bf16",
            "gff_gemm_bf16_strided", "gff_gemm_bf16_workspace_bytes", "gff_gather_rows", "gff_relax_graph_create",
            "gff_graph_launch", "gff_graph_destroy", "gff_autotune",
            "gff_refill", "gff_dedupe_rmsd", "gff_dedupe_rmsd_workspace_bytes", "gff_dedupe_rmsd_noalloc",
            "gff_gather_probe"]
N_ENC = 41


def _rt(name, restype):
    getattr(lib(), name).restype = restype


def propose_uniform(n_rep, n_tors, seed, rnd, h_lo, h_hi, d_dof, d_raw=None, stream=None):
    check(lib().gff_propose_uniform(C.c_int(n_rep), C.c_int(n_tors), C.c_uint64(seed), C.c_uint32(rnd),
                                    C.c_float(h_lo), C.c_float(h_hi), _ptr(d_dof), _ptr(d_raw), _stream(stream)))


def refill(plan, d_mode, d_pos_src, st, dt0=0.05, alpha0=0.1, stream=None):
    """Replace (mode 1) or freeze (mode 2) replicas of a relaxation state between launches."""
    state = _state(st)
    check(lib().gff_refill(plan.handle, _ptr(d_mode), _ptr(d_pos_src), C.c_float(dt0), C.c_float(alpha0),
                           C.byref(state), _stream(stream)))


def pose_from_dof(topo, plan, d_dof, dof_stride, Lx, Ly, z_top, d_pos, stream=None):
    check(lib().gff_pose_from_dof(topo.handle, plan.handle, _ptr(d_dof), C.c_int(dof_stride), C.c_float(Lx),
                                  C.c_float(Ly), C.c_float(z_top), _ptr(d_pos), _stream(stream)))


def encode_pose(topo, plan, d_pos, Lx, Ly, z_top, d_work, d_enc, stream=None):
    check(lib().gff_encode_pose(topo.handle, plan.handle, _ptr(d_pos), C.c_float(Lx), C.c_float(Ly), C.c_float(z_top),
                                _ptr(d_work), _ptr(d_enc), _stream(stream)))


def decode_dof(d_enc, n_tors, h_lo, h_hi, d_dof, stream=None):
    check(lib().gff_decode_dof(C.c_int(d_enc.shape[0]), _ptr(d_enc), C.c_int(n_tors), C.c_float(h_lo),
                               C.c_float(h_hi), _ptr(d_dof), _stream(stream)))


def dedupe_energy(d_E, d_type, d_ok, tol, capacity, d_arch_E, d_arch_type, d_arch_n, d_is_new, stream=None):
    check(lib().gff_dedupe_energy(C.c_int(d_E.numel()), _ptr(d_E), _ptr(d_type), _ptr(d_ok), C.c_double(tol),
                                  C.c_int(capacity), _ptr(d_arch_E), _ptr(d_arch_type), _ptr(d_arch_n),
                                  _ptr(d_is_new), _stream(stream)))


def dedupe_rmsd_workspace_bytes(n_rep):
    return lib().gff_dedupe_rmsd_workspace_bytes(C.c_int(n_rep))


def dedupe_rmsd(plan, d_pos, d_ok, tol, Lx, Ly, capacity, max_atoms, d_arch_pos, d_arch_cen, d_arch_type, d_arch_n,
                d_is_new, d_work=None, stream=None):
    """d_work: device scratch of dedupe_rmsd_workspace_bytes(plan.n_rep) bytes (allocated
    here when not given)."""
    nb = dedupe_rmsd_workspace_bytes(plan.n_rep)
    if d_work is None and nb > 0:
        import torch
        d_work = torch.empty(nb, dtype=torch.uint8, device=d_is_new.device)
    check(lib().gff_dedupe_rmsd(plan.handle, _ptr(d_pos), _ptr(d_ok), C.c_float(tol), C.c_float(Lx), C.c_float(Ly),
                                C.c_int(capacity), C.c_int(max_atoms), _ptr(d_arch_pos), _ptr(d_arch_cen),
                                _ptr(d_arch_type), _ptr(d_arch_n), _ptr(d_is_new), _ptr(d_work),
                                C.c_size_t(0 if d_work is None else d_work.numel() * d_work.element_size()),
                                _stream(stream)))


DEDUPE_NOALLOC_MAX_REP = 65536


def dedupe_rmsd_noalloc(plan, d_pos, d_ok, tol, Lx, Ly, capacity, max_atoms, d_arch_pos, d_arch_cen, d_arch_type,
                        d_arch_n, d_is_new, stream=None):
    """dedupe_rmsd with the library's static scratch (no allocation anywhere in the call)."""
    check(lib().gff_dedupe_rmsd_noalloc(plan.handle, _ptr(d_pos), _ptr(d_ok), C.c_float(tol), C.c_float(Lx),
                                        C.c_float(Ly), C.c_int(capacity), C.c_int(max_atoms), _ptr(d_arch_pos),
                                        _ptr(d_arch_cen), _ptr(d_arch_type), _ptr(d_arch_n), _ptr(d_is_new),
                                        _stream(stream)))


def normal_philox(n, seed, rnd, d_out, stream=None):
    check(lib().gff_normal_philox(C.c_long(n), C.c_uint64(seed), C.c_uint32(rnd), _ptr(d_out), _stream(stream)))


def gemm_bf16(d_A, d_B, d_C, stream=None):
    M, K = d_A.shape
    N = d_B.shape[1]
    check(lib().gff_gemm_bf16(C.c_int(M), C.c_int(N), C.c_int(K), _ptr(d_A), _ptr(d_B), _ptr(d_C), _stream(stream)))


def gemm_bf16_workspace_bytes():
    L = lib()
    L.gff_gemm_bf16_workspace_bytes.restype = C.c_size_t
    return L.gff_gemm_bf16_workspace_bytes()


def gemm_bf16_strided(M, N, K, d_A, sam, sak, d_B, sbk, sbn, d_C, ldc, d_work=None, stream=None):
    """C[m*ldc + n] = sum_k A[m*sam + k*sak] B[k*sbk + n*sbn] (element strides; BF16 words in
    int16 tensors, FP32 out); with d_work (uint8, gemm_bf16_workspace_bytes()) K may split."""
    check(lib().gff_gemm_bf16_strided(C.c_int(M), C.c_int(N), C.c_int(K), _ptr(d_A), C.c_long(sam), C.c_long(sak),
                                      _ptr(d_B), C.c_long(sbk), C.c_long(sbn), _ptr(d_C), C.c_long(ldc),
                                      _ptr(d_work),
                                      C.c_size_t(0 if d_work is None else d_work.numel() * d_work.element_size()),
                                      _stream(stream)))


def gather_probe(d_buf, n_threads, iters, seed, d_sink, stream=None):
    """Random 64-byte-chunk gather over the bytes of d_buf (see gff_gather_probe)."""
    check(lib().gff_gather_probe(_ptr(d_buf), C.c_size_t(d_buf.numel() * d_buf.element_size()),
                                 C.c_int(n_threads), C.c_int(iters), C.c_uint(seed), _ptr(d_sink),
                                 _stream(stream)))


def imle_select(d_cand, d_target, d_ntors, d_best, d_bestd=None, stream=None):
    n, K = d_cand.shape[0], d_cand.shape[1]
    check(lib().gff_imle_select(C.c_int(n), C.c_int(K), _ptr(d_cand), _ptr(d_target), _ptr(d_ntors), _ptr(d_best),
                                _ptr(d_bestd), _stream(stream)))


class MLP:
    """The learned proposer (device-resident FP32 masters, BF16 copies, Adam moments)."""

    def __init__(self, n_types, params):
        L = lib()
        L.gff_mlp_n_params.restype = C.c_size_t
        L.gff_mlp_workspace_bytes.restype = C.c_size_t
        self.n_types = n_types
        self.n_params = L.gff_mlp_n_params(C.c_int(n_types))
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == self.n_params, (p.size, self.n_params)
        self.handle = C.c_void_p()
        check(L.gff_mlp_create(C.c_int(n_types), p.ctypes.data_as(C.c_void_p), C.byref(self.handle)))
        self._work = None

    def workspace(self, batch):
        import torch
        need = lib().gff_mlp_workspace_bytes(C.c_int(batch))
        if self._work is None or self._work.numel() < need:
            self._work = torch.empty(need, dtype=torch.uint8, device="cuda")
        return self._work

    def params(self):
        p = np.zeros(self.n_params, np.float32)
        g = np.zeros(self.n_params, np.float32)
        check(lib().gff_mlp_get_params(self.handle, p.ctypes.data_as(C.c_void_p), g.ctypes.data_as(C.c_void_p)))
        return p, g

    def forward(self, d_noise, d_type, d_out, stream=None):
        B = d_noise.shape[0]
        w = self.workspace(B)
        check(lib().gff_mlp_forward(self.handle, C.c_int(B), _ptr(d_noise), _ptr(d_type), _ptr(d_out), _ptr(w),
                                    C.c_size_t(w.numel()), _stream(stream)))

    def train_step(self, d_noise, d_type, d_target, d_ntors, lr, d_out, d_loss=None, stream=None):
        B = d_noise.shape[0]
        w = self.workspace(B)
        check(lib().gff_mlp_train_step(self.handle, C.c_int(B), _ptr(d_noise), _ptr(d_type), _ptr(d_target),
                                       _ptr(d_ntors), C.c_float(lr), _ptr(d_out), _ptr(d_loss), _ptr(w),
                                       C.c_size_t(w.numel()), _stream(stream)))

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.gff_mlp_destroy(self.handle)
            self.handle = None


def gather_rows(d_src, K, d_idx, d_dst, stream=None):
    n, ln = d_dst.shape[0], d_dst.shape[-1]
    check(lib().gff_gather_rows(C.c_int(n), C.c_int(ln), _ptr(d_src), C.c_int(K), _ptr(d_idx), _ptr(d_dst),
                                _stream(stream)))


class RelaxGraph:
    """A captured relaxation launch (fixed buffers); launch() re-runs it."""

    def __init__(self, grid_desc, topo, plan, params, st, d_E_rep, d_fnorm, d_steps, d_drift=None):
        self.state = _state(st)
        self.keep = (grid_desc, topo, plan, params, st, d_E_rep, d_fnorm, d_steps, d_drift)
        self.handle = C.c_void_p()
        check(lib().gff_relax_graph_create(C.byref(grid_desc), topo.handle, plan.handle, C.byref(params),
                                           C.byref(self.state), _ptr(d_E_rep), _ptr(d_fnorm), _ptr(d_steps),
                                           _ptr(d_drift), C.byref(self.handle)))

    def launch(self, stream=None):
        check(lib().gff_graph_launch(self.handle, _stream(stream)))

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.gff_graph_destroy(self.handle)
            self.handle = None


def autotune(grid_desc, topo, rep_type, params, st, stream=None):
    """Measured launch shape -> (Launch, replica-steps/s)."""
    rt = np.ascontiguousarray(rep_type, dtype=np.int32)
    state = _state(st)
    best = Launch()
    rate = C.c_float()
    check(lib().gff_autotune(C.byref(grid_desc), topo.handle, C.c_int(len(rt)), rt.ctypes.data_as(C.c_void_p),
                             C.byref(params), C.byref(state), C.byref(best), C.byref(rate), _stream(stream)))
    return best, rate.value
