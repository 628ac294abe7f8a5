/*
 * gridff.h -- C ABI of the MI355X (gfx950) GridFF hot path.
 *
 * GridFF (Mal, Koci, Nicolini & Hapala, arXiv 2508.15522) replaces the molecule-
 * substrate interaction by three precomputed grids -- Pauli V^P, London V^L and
 * Coulomb V^C -- that carry no molecular types or charges (Section "Principles",
 * Eqs. E, E_Coulomb, E_Morse, V_Morse).  Each atom's energy is the tricubic
 * B-spline interpolant of the grids mixed with the atom's own coefficients,
 *     E_i = P_i V^P(r_i) + L_i V^L(r_i) + Q_i V^C(r_i),
 *     P_i = eps_i exp(2 alpha R_i),  L_i = -2 eps_i exp(alpha R_i),  Q_i = charge,
 * and forces are the analytic gradient of that interpolant (Section
 * "Interpolation", Eqs. Bspline1D, Bspline).  The library builds the grids,
 * fits the B-spline coefficients, evaluates energies and forces, and relaxes
 * (FIRE) or integrates (velocity-Verlet NVE) thousands of independent molecule
 * replicas at once, with the whole step loop on the GPU (Section "Configuration
 * sampling on GPU").
 *
 * Conventions for every entry point:
 *  - Units: energy eV, length Angstrom, charge e, mass amu, time fs (NVE) or the
 *    unit-mass FIRE time unit.
 *  - Pointers named d_* are device memory owned by the caller; *_h pointers are
 *    host memory owned by the caller.  Opaque handles (gff_topology, gff_plan) own
 *    device memory they allocate at creation and free on destroy.  No entry point
 *    that takes a stream allocates device memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Calls
 *    only enqueue work; outputs are valid once the stream has synchronised.
 *  - Arguments are validated before anything is enqueued; a negative gff_status
 *    means nothing was enqueued.  GFF_EHIP reports a HIP launch/runtime error.
 *  - Per-replica physics problems are not errors: they are GFF_REP_* status bits.
 *  - Results are deterministic: identical inputs give bitwise-identical outputs
 *    (no floating-point atomics; every reduction has a fixed order).
 *  - Per-atom arrays are structure-of-arrays [3][n_atoms_total] (x block, then y,
 *    then z).  Replica r owns atoms atom_off[r] .. atom_off[r+1]-1 where atom_off is
 *    the prefix sum of the replicas' atom counts in replica order.
 */
#ifndef GRIDFF_H
#define GRIDFF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GFF_OK = 0,
    GFF_EINVAL = -1,          /* invalid argument (null pointer, bad size, inconsistent grid) */
    GFF_EUNSUPPORTED = -2,    /* valid request the library does not implement (e.g. > 128 atoms) */
    GFF_EHIP = -3,            /* HIP runtime or launch error */
    GFF_EWORKSPACE = -4,      /* workspace smaller than the *_workspace_bytes query */
    GFF_ENOMEM = -5           /* allocation failed inside a create call */
} gff_status;

enum { GFF_STORE_F32 = 0, GFF_STORE_F16 = 1, GFF_STORE_TRILINEAR = 2 };

/* per-replica status bits */
enum {
    GFF_REP_CONVERGED = 1,     /* FIRE: |F|_2 over the replica's 3N force vector < f_conv; frozen */
    GFF_REP_OUT_OF_DOMAIN = 2, /* an atom was below the first grid plane (evaluated on that plane) */
    GFF_REP_NONFINITE = 4,     /* a non-finite force/energy/coordinate appeared; replica frozen */
    GFF_REP_MAXSTEPS = 8       /* FIRE with f_conv > 0 ended without converging */
};

enum { GFF_MODE_FIRE = 0, GFF_MODE_NVE = 1, GFF_MODE_LANGEVIN = 2 };

const char *gff_status_string(int status);

/* ------------------------------------------------------------------ grid build and fit */

/* Rigid substrate, host FP64, periodic in x and y with an orthorhombic Lx x Ly cell.
 * The lateral periodicity is the substrate's only (Section "Periodicity and long-range
 * electrostatics"): the molecule never meets its own images. */
typedef struct {
    int n_atoms;
    const double *pos_h;   /* [n_atoms][3] */
    const double *q_h;     /* [n_atoms] charges; the slab must be neutral with zero z-dipole */
    const double *eps_h;   /* [n_atoms] Morse eps_j (pair depth eps_i eps_j) */
    const double *R_h;     /* [n_atoms] Morse R_j (pair separation R_i + R_j) */
    double Lx, Ly;
} gff_substrate;

/* Grid geometry and build physics.  Node (i,j,k) sits at
 * (x0 + i Lx/nx, y0 + j Ly/ny, z0 + k dz); x and y are periodic, so the node spacing is
 * dx = Lx/nx, dy = Ly/ny.  z0 must lie above every substrate atom (the Coulomb channel is
 * built with the above-slab Fourier form of the 2D lattice sum). */
typedef struct {
    int nx, ny, nz;          /* >= 4 each */
    double x0, y0, z0, dz;
    double alpha;            /* Morse alpha [1/A] (the paper uses one alpha for all pairs) */
    double rcut;             /* direct-sum cutoff of the Pauli/London image sums [A] */
    double k_e;              /* Coulomb constant; <= 0 selects 14.3996454784 eV A/e^2 */
} gff_grid_spec;

/* V[c][i][j][k], c = 0 Pauli, 1 London, 2 Coulomb, FP64, z fastest:
 *   V^P(r) = sum_j sum_n eps_j exp(-2 alpha(|r - r_j - n| - R_j))   (images n, |.| < rcut)
 *   V^L(r) = sum_j sum_n eps_j exp(-alpha(|r - r_j - n| - R_j))
 *   V^C(r) = k_e sum_{G != 0} (2 pi / A) sum_j Q_j cos(G.(rho - rho_j)) exp(-|G|(z - z_j)) / |G|
 * (Eq. V_Morse; Section "Periodicity and long-range electrostatics": the exact
 * 2D-periodic Coulomb lattice sum above a neutral zero-dipole slab, V^C -> 0 far above;
 * the paper's reciprocal-space Poisson solve approximates the same potential).
 * d_work: at least gff_build_grid_workspace_bytes(spec, sub) bytes of device memory. */
size_t gff_build_grid_workspace_bytes(const gff_grid_spec *spec, const gff_substrate *sub);
gff_status gff_build_grid(const gff_substrate *sub, const gff_grid_spec *spec, double *d_V,
                          void *d_work, size_t work_bytes, void *stream);

/* Exact B-spline coefficients B[3][nx][ny][nz] (FP64) of V[3][nx][ny][nz]: the tricubic
 * B-spline model reproduces V at every node (Section "Interpolation", fitting paragraph;
 * the paper fits this linear system by gradient descent, here it is solved exactly by
 * separable tridiagonal solves: cyclic along x and y, even-mirror rows along z, i.e.
 * (4 b_0 + 2 b_1)/6 = V_0 and (2 b_{n-2} + 4 b_{n-1})/6 = V_{n-1}).  d_B may not alias d_V.
 * d_work: gff_fit_workspace_bytes(spec) bytes. */
size_t gff_fit_workspace_bytes(const gff_grid_spec *spec);
gff_status gff_fit_bspline(const gff_grid_spec *spec, const double *d_V, double *d_B,
                           void *d_work, size_t work_bytes, void *stream);

/* Storage cast of fitted coefficients into the evaluation layout:
 * coef[i][j][b][r][c4], padded z plane p = 0 .. nz+2 holding z node p-1 with even-mirror
 * padding (node -1 -> 1, node nz -> nz-2, node nz+1 -> nz-3), c4 = (Pauli, London,
 * Coulomb, 0) (F16: (Pauli, London, Coulomb, Pauli residual)).  Each column is stored as
 * (nz-1)/5 + 1 overlapping z blocks of 8 slots: slot r of block b holds plane 5b + r (zero
 * past plane nz+2).  The four planes k .. k+3 an interpolation in z cell k reads are slots
 * k mod 5 .. k mod 5 + 3 of block k / 5, one 128-byte (F32) or 64-byte (F16) aligned unit
 * when d_coef is 128-byte aligned, which keeps every column read inside one cache line.
 * GFF_STORE_F32: float; GFF_STORE_F16: IEEE half h_c of b_c / s_c (round to nearest even),
 * with per-channel scale s_c = 2^(ceil(log2 max|b_c|) - 15) written to d_scale[0..2]
 * (d_scale[3] = 0); the fourth half holds l = half(b_P / s_P - h_P), the rounding residual
 * of the Pauli channel, whose mixed values dominate the force near the surface, and the
 * evaluation decodes Pauli as (h_P + l) s_P (8 bytes per node either way).  For F32,
 * d_scale (if not NULL) receives 1,1,1,0.
 * GFF_STORE_TRILINEAR, the earlier scheme the paper compares against (Section
 * "Interpolation": energy and force stored per node and interpolated trilinearly, each on
 * its own): tri[i][j][k][c] = float4 (E, dE/du, dE/dv, dE/dw) of channel c, the fitted
 * model's value and gradient with respect to the node-index coordinates u = (x - x0)/dx,
 * v, w at node (i, j, k), formed in FP64 from the coefficients (even-mirror rows at the z
 * ends) and stored in FP32, 48 bytes per node (the evaluation scales the interpolated
 * gradient by -1/dx, -1/dy, -1/dz into a force); d_scale as for F32.
 * d_coef: gff_grid_bytes(spec, storage) bytes. */
size_t gff_grid_bytes(const gff_grid_spec *spec, int storage);
gff_status gff_pack_grid(const gff_grid_spec *spec, const double *d_B, int storage,
                         void *d_coef, float *d_scale, void *stream);

/* ------------------------------------------------------------------ evaluation */

/* A fitted, device-resident grid in the gff_pack_grid layout.  The lateral period is
 * nx*dx by ny*dy.  Coordinates below z0 are evaluated on the z0 plane (and flagged);
 * coordinates strictly above the last node z0 + (nz-1) dz contribute zero.  A
 * GFF_STORE_TRILINEAR grid interpolates the stored nodal energy and force of each channel
 * trilinearly in the cell, mixed with the atom's (P, L, Q); its force is therefore not the
 * gradient of its energy.  F32 and F16 grids are read through 32-bit buffer offsets: a grid
 * of gff_grid_bytes >= 4 GiB - 1 is rejected with GFF_EUNSUPPORTED by every call that
 * evaluates it (a trilinear table needs nx*ny*nz < 2^31). */
typedef struct {
    int storage;             /* GFF_STORE_F32, GFF_STORE_F16 or GFF_STORE_TRILINEAR */
    int nx, ny, nz;
    float x0, y0, z0, dx, dy, dz;
    const void *d_coef;
    const float *d_scale;    /* [4] decode scale (F16); NULL for F32 means 1 */
} gff_grid;

/* One molecule type, host arrays, FP32.  Intramolecular field (synthetic, explicit):
 *   bond 1/2 k (r - r0)^2; angle 1/2 k (cos th - cos0)^2 (vertex = middle index);
 *   torsion 1/2 V (1 - cos(n phi - phi0)), phi the IUPAC dihedral of (i,j,k,l);
 *   non-bonded for pairs more than two bonds apart: Morse with depth eps_i eps_j at
 *   R_i + R_j and the grid's alpha, plus k_e Q_i Q_j / r.
 * The rotatable torsions (rot_quads, rot_mask) and ref_pos are only used by pose
 * construction and may be empty/NULL otherwise. */
typedef struct {
    int n_atoms;                         /* 1 .. 128 */
    const float *eps, *R, *q, *mass;     /* [n_atoms] */
    int n_bonds;  const int *bonds;  const float *bond_k, *bond_r0;       /* bonds [n][2] */
    int n_angles; const int *angles; const float *angle_k, *angle_cos0;  /* angles [n][3] */
    int n_tors;   const int *tors;   const float *tors_V; const int *tors_n; const float *tors_phi0; /* [n][4] */
    int n_rot;    const int *rot_quads; const unsigned char *rot_mask;   /* [n_rot][4], [n_rot][n_atoms] */
    const float *ref_pos;                /* [n_atoms][3] reference geometry */
} gff_mol_type;

typedef struct gff_topology_s gff_topology;

/* Builds the device tables of a set of molecule types (mixing coefficients P, L, Q from
 * (eps, R, q) and alpha; per-atom incidence lists of bonded terms; 1-2/1-3 exclusion
 * masks).  Allocates device memory; not stream-ordered (synchronous upload). */
gff_status gff_topology_create(const gff_mol_type *types_h, int n_types, float alpha, float k_e,
                               gff_topology **out);
void gff_topology_destroy(gff_topology *topo);

/* Launch shape of the replica kernels.  block_threads: multiple of 64 in [64, 1024];
 * replicas of one type are packed densely into blocks, lanes_per_atom lanes per atom (1, 2
 * or 4; 0 means 1), floor(block / (lanes_per_atom n)) replicas per block (at most
 * reps_per_block if > 0).  grid_blocks <= 0: one block per pack.  Several lanes per atom
 * split an atom's non-bonded partners, bonded terms and the replica's torsion terms (and,
 * at four, give every atom its own gather quad): for batches too small to fill the GPU and
 * for batches of large molecules, whose pair work per lane grows with the molecule.
 * They apply to FIRE, NVE and Langevin launches on FP32 and FP16 B-spline grids; other
 * launches on such a plan use one lane per atom on the same packing.  Results depend on
 * lanes_per_atom only through the FP32 summation order of the split sums. */
typedef struct {
    int block_threads;
    int reps_per_block;
    int grid_blocks;
    int lanes_per_atom;
} gff_launch;

typedef struct gff_plan_s gff_plan;

/* Work list for a batch of n_rep replicas with types rep_type_h[r]: packs of same-type
 * replicas, sorted largest type first.  Allocates device memory (synchronous). */
gff_status gff_plan_create(const gff_topology *topo, int n_rep, const int *rep_type_h,
                           const gff_launch *launch /* NULL = default */, gff_plan **out);
void gff_plan_destroy(gff_plan *plan);
int gff_plan_n_atoms(const gff_plan *plan);
int gff_plan_n_packs(const gff_plan *plan);
/* atom_off_h[n_rep+1]: the replica atom offsets of the per-atom arrays */
gff_status gff_plan_atom_offsets(const gff_plan *plan, int *atom_off_h);

/* Energy and forces at fixed positions.  The grid part is the per-atom tricubic B-spline
 * interpolation of the three channels mixed with the atom's (P, L, Q) (Section
 * "Interpolation", Eqs. Bspline1D and Bspline; Section "Principles", Eqs. E, E_Morse,
 * E_Coulomb and V_Morse: E_i = P_i V^P + L_i V^L + Q_i V^C, F_i = -grad E_i); the
 * intramolecular field is the force field the paper takes from UFF (Section "Accuracy and
 * performance tests on CPU"), here with the explicit terms documented with gff_mol_type.
 * d_F [3][N] = -grad E (grid part plus, if include_intra, the intramolecular field);
 * d_E_atom [N] (nullable) the per-atom grid energy E_i; d_E_rep [n_rep] (nullable) the
 * replica's total energy, summed in FP64; d_status [n_rep] (nullable) OUT_OF_DOMAIN /
 * NONFINITE bits. */
gff_status gff_eval_forces(const gff_grid *grid, const gff_topology *topo, const gff_plan *plan,
                           int include_intra, const float *d_pos, float *d_F, float *d_E_atom,
                           double *d_E_rep, unsigned *d_status, void *stream);

/* Plain per-point interpolation (no molecules): d_pos [3][n], d_plq [3][n] = (P, L, Q)
 * per point, outputs d_F [3][n] and d_E [n] (nullable). */
gff_status gff_interp_points(const gff_grid *grid, int n, const float *d_pos, const float *d_plq,
                             float *d_F, float *d_E, void *stream);

/* ------------------------------------------------------------------ relaxation / dynamics */

typedef struct {
    int mode;                 /* GFF_MODE_FIRE, GFF_MODE_NVE or GFF_MODE_LANGEVIN */
    int n_steps;              /* moves (FIRE) or time steps (NVE, Langevin); >= 0 */
    int include_intra;
    float dt;                 /* NVE/Langevin time step [fs]; FIRE: unused (per-replica dt is state) */
    float f_conv;             /* FIRE convergence on |F|_2 [eV/A]; <= 0: never */
    float max_disp;           /* FIRE per-atom displacement cap per step [A] */
    float fire_finc, fire_fdec, fire_alpha0, fire_falpha, fire_dtmax;
    int fire_nmin;
    int drift_every;          /* NVE: FP64 total-energy sample every k steps (>= 1) */
    float kT;                 /* Langevin: bath temperature k_B T [eV] (>= 0) */
    float gamma;              /* Langevin: friction [1/fs] (>= 0) */
    unsigned long long seed;  /* Langevin: Philox key (low word, high word) */
    unsigned round;           /* Langevin: fourth Philox counter word; use a new value per launch */
    int check_every;          /* FIRE: replica-wide decisions every k-th move (the paper's GPU
                                 sampler checks every 100 steps); 0 or 1: every move */
} gff_relax_params;

/* Caller-owned replica state (in/out). */
typedef struct {
    float *d_pos;             /* [3][N] */
    float *d_vel;             /* [3][N]; FIRE: unit-mass velocities, NVE: A/fs */
    float *d_fire_dt;         /* [n_rep] FIRE time step (initialise to dt0) */
    float *d_fire_alpha;      /* [n_rep] FIRE mixing (initialise to alpha0) */
    int *d_fire_npos;         /* [n_rep] steps since P <= 0 (initialise to 0) */
    unsigned *d_status;       /* [n_rep] GFF_REP_* bits (initialise to 0) */
    /* Restraint, FIRE only (the manipulation scans of Sections "Relaxed detachment" and
     * "Dragging": one atom held, the rest relaxed); both NULL for none.  d_fixed_atom [n_rep]:
     * index of the held atom in its molecule (outside [0, n): none); d_fixed_pos [n_rep][3]:
     * where it is held.  On entry the atom is placed there with zero velocity; its force is
     * replaced by zero, so it never moves and takes no part in |F|_2, P = F.v or the mixing;
     * the energy is the whole replica's. */
    const int *d_fixed_atom;
    const float *d_fixed_pos;
} gff_state;

/* Batched relaxation and dynamics of independent replicas, the whole step loop in one
 * launch (Section "Configuration sampling on GPU": many replicas at once, the MD loop kept on
 * the GPU; the energy and forces are those of gff_eval_forces).
 *
 * FIRE (Bitzek et al. 2006; the relaxation of Sections "Accuracy and performance tests on
 * CPU" and "Configuration sampling on GPU") per replica with unit masses, every step on the
 * GPU: evaluate F, E at x; if |F|_2 < f_conv set CONVERGED and freeze; P = F.v;
 * v <- (1-a) v + a |v| F/|F|; if P > 0 { npos++; if npos > nmin: dt <- min(dt finc, dtmax),
 * a <- a falpha } else { dt <- dt fdec; a <- alpha0; v <- 0; npos <- 0 }; v <- v + F dt;
 * dx = v dt scaled per atom to |dx_i| <= max_disp; x <- x + dx.  After n_steps moves the
 * final state is evaluated once more.  Replicas converged on entry are evaluated, not moved.
 * With check_every = k > 1 (the paper's form, which downloads the state every 100 steps to
 * test convergence and stop uphill motion) the steps that need sums over the replica (the
 * convergence test, P, mixing, adaptation, restart) are taken only on moves 0, k, 2k, ... and
 * at the final evaluation; the moves in between are plain kicks v <- v + F dt with capped
 * moves at the current dt.  Not supported by gff_relax_scan (GFF_EINVAL).
 *
 * NVE: velocity Verlet with masses in amu, a = F/(m 103.6427) [A/fs^2]; forces at the
 * entry positions are evaluated first.  Every drift_every steps the total energy
 * E_pot + sum m v^2/2 is formed in FP64 and accumulated in d_drift_rep[r][6] =
 * {E(0), E(last sample), max|E(s)-E(0)|, sum dE, sum s dE, samples}; non-finite energies
 * freeze the replica at those samples.
 *
 * Langevin (the thermal perturbation of minima hopping, Section "Configuration sampling on
 * GPU"; the paper names no integrator, this is BAOAB, Leimkuhler & Matthews 2013): per step
 * v += dt/2 a; x += dt/2 v; v <- c1 v + c2 sqrt(kT/m) xi; x += dt/2 v; a = a(x); v += dt/2 a,
 * c1 = exp(-gamma dt), c2 = sqrt(1 - c1^2), masses as in NVE.  The three normals xi of
 * replica r (its index in the plan), atom a of the molecule and step s = 1..n_steps come
 * from Philox4x32-10 with counter (r, a, s, round) and key (seed low, seed high): with
 * u_k = ((x_k >> 9) + 1/2) 2^-23, xi = (sqrt(-2 ln u0) cos 2pi u1, sqrt(-2 ln u0) sin 2pi u1,
 * sqrt(-2 ln u2) cos 2pi u3).  d_drift_rep must be NULL; d_fnorm_rep receives 0.  A replica
 * whose coordinates become non-finite ends with GFF_REP_NONFINITE and a NaN energy; its
 * final positions are unspecified.
 *
 * Outputs: d_E_rep [n_rep] (FP64 total energy at the last evaluation), d_fnorm_rep
 * [n_rep] (|F|_2 there, FP32), d_steps_rep [n_rep] (moves made), d_drift_rep nullable.
 * One kernel launch runs the whole step loop.  The FIRE loop forms forces only; when
 * d_E_rep is given, a second launch evaluates the energies at the final positions (those of
 * the last evaluation: a converged replica stops moving). */
gff_status gff_relax_batch(const gff_grid *grid, const gff_topology *topo, const gff_plan *plan,
                           const gff_relax_params *params, const gff_state *state,
                           double *d_E_rep, float *d_fnorm_rep, int *d_steps_rep,
                           double *d_drift_rep, void *stream);

/* A whole restrained scan in one launch (Sections "Relaxed detachment" and "Dragging": the
 * held atom moved point by point, the rest relaxed at each point, continuing from the
 * previous point).  FIRE only (params->mode == GFF_MODE_FIRE; params->n_steps is ignored);
 * state->d_fixed_atom names each replica's held atom (state->d_fixed_pos is not used).  Per
 * replica r the held atom is placed at d_path[r][p] (float [n_rep][n_points][3]) for
 * p = 0 .. n_points-1; at each point FIRE runs until |F|_2 < f_conv or moves_per_point moves,
 * then the point's energy (FP32 sum over the replica's atoms), move count, status
 * (GFF_REP_CONVERGED or GFF_REP_MAXSTEPS) and optionally all positions are recorded and FIRE
 * restarts for the next point (velocities 0, dt = dt0, alpha = fire_alpha0, count 0).  Each
 * replica advances on its own, so a launch costs the slowest replica's total moves rather
 * than the sum over points of each point's slowest replica.  The trajectory of every replica
 * is that of one gff_relax_batch launch per point with a gff_refill restart in between.
 * Outputs: d_E_points [n_rep][n_points] (FP64 holding the FP32 sums), d_steps_points and
 * d_status_points [n_rep][n_points] (nullable), d_pos_points [n_points][3][N] (nullable),
 * and as gff_relax_batch the final state, d_E_rep, d_fnorm_rep, d_steps_rep (total moves).
 * A replica that enters with GFF_REP_CONVERGED or GFF_REP_NONFINITE set, or becomes
 * non-finite during the scan, is not scanned further: its remaining per-point entries are
 * left unwritten (initialise the status with 0 to scan every replica). */
gff_status gff_relax_scan(const gff_grid *grid, const gff_topology *topo, const gff_plan *plan,
                          const gff_relax_params *params, const gff_state *state, const float *d_path, int n_points,
                          int moves_per_point, float dt0, double *d_E_points, int *d_steps_points,
                          unsigned *d_status_points, float *d_pos_points, double *d_E_rep, float *d_fnorm_rep,
                          int *d_steps_rep, void *stream);

/* ------------------------------------------------------------------ all-atom comparison mode */

/* The all-atom molecule-substrate evaluation that the paper compares GridFF with (Section
 * "Configuration sampling on GPU"): every substrate atom of the cell and of its lateral
 * periodic images (a, b), |a|, |b| <= n_img (n_img = 1: the cell and its 8 neighbours, 9
 * cells), summed directly per molecule atom with no cutoff and bare Coulomb:
 *   E_i = sum_j sum_ab [ P_i eps_j e^{2 alpha R_j} e^{-2 alpha r} + L_i eps_j e^{alpha R_j} e^{-alpha r}
 *                        + k_e Q_i q_j / r ].
 * gff_direct_create uploads the substrate (synchronous; allocates device memory); alpha must
 * equal the topology's.  gff_eval_forces_direct and gff_relax_batch_direct take the place
 * of gff_eval_forces and gff_relax_batch with the grid replaced by this sum; everything
 * else (intramolecular field, FIRE, NVE, outputs, status flags) is the same.  Errors as
 * for those calls; GFF_EINVAL also when alpha differs from the topology's. */
typedef struct gff_direct_s gff_direct;
gff_status gff_direct_create(const gff_substrate *sub, float alpha, int n_img, gff_direct **out);
void gff_direct_destroy(gff_direct *direct);
gff_status gff_eval_forces_direct(const gff_direct *direct, const gff_topology *topo, const gff_plan *plan,
                                  int include_intra, const float *d_pos, float *d_F, float *d_E_atom,
                                  double *d_E_rep, unsigned *d_status, void *stream);
gff_status gff_relax_batch_direct(const gff_direct *direct, const gff_topology *topo, const gff_plan *plan,
                                  const gff_relax_params *params, const gff_state *state, double *d_E_rep,
                                  float *d_fnorm_rep, int *d_steps_rep, double *d_drift_rep, void *stream);

/* Resident blocks per compute unit of the kernel gff_relax_batch (mode GFF_MODE_FIRE or
 * GFF_MODE_NVE) or gff_eval_forces (mode -1) launches for this grid storage and plan,
 * from the device's occupancy calculator (register and LDS limits); *lds_bytes_out
 * (nullable) receives the dynamic LDS of one block.  GFF_EINVAL on null arguments or
 * an unknown mode. */
gff_status gff_relax_occupancy(const gff_grid *grid, const gff_plan *plan, int mode, int *blocks_per_cu,
                               size_t *lds_bytes_out);

/* ------------------------------------------------------------------ graphs and autotuning */

/* One relaxation launch captured as a HIP graph (arguments and buffers fixed at capture);
 * every gff_graph_launch re-runs it on the same buffers, continuing from their current
 * contents.  The graph holds no memset nodes. */
typedef struct gff_graph_s gff_graph;
gff_status gff_relax_graph_create(const gff_grid *grid, const gff_topology *topo, const gff_plan *plan,
                                  const gff_relax_params *params, const gff_state *state, double *d_E_rep,
                                  float *d_fnorm_rep, int *d_steps_rep, double *d_drift_rep, gff_graph **out);
gff_status gff_graph_launch(gff_graph *graph, void *stream);
void gff_graph_destroy(gff_graph *graph);

/* Measured launch shape for a batch (setup step: allocates scratch and synchronises): runs
 * `params` for every block size 64..1024 (multiple of 64, >= the largest molecule) with the
 * densest packing and, when that gives fewer than two packs per compute unit, with at most
 * 1, 2, 4 or 8 replicas per block; each with the default grid and with persistent grids of
 * 1-4 blocks per compute unit; on FP32/FP16 B-spline grids all of this again with 2 lanes
 * per atom and, for batches of fewer atoms than 256 per compute unit, with 4 (Section
 * "Configuration sampling on GPU": the GPU has far more cores than a small molecule has
 * atoms, and a large molecule's pair work splits across lanes); on copies of `state`;
 * returns the fastest shape and its replica-steps/s (nullable). */
gff_status gff_autotune(const gff_grid *grid, const gff_topology *topo, int n_rep, const int *rep_type_h,
                        const gff_relax_params *params, const gff_state *state, gff_launch *best,
                        float *best_rate, void *stream);

/* ------------------------------------------------------------------ proposals and minima */

/* Degrees of freedom per replica, float [n][7 + T]: u, v (lateral centroid as fractions of the
 * cell), h (height of the lowest atom above z_top), unit quaternion (w, x, y, z) of the rigid
 * rotation about the centroid, and T target dihedrals (IUPAC) of the rotatable torsions.
 * The sampling loop perturbs poses and relaxes them to nearby minima (Section
 * "Configuration sampling on GPU"); here proposals are drawn directly. */

/* Uniform proposals from Philox4x32-10 (Salmon et al. 2011) with counter (replica, block,
 * round, 0) and key (seed low, seed high): block 0 gives (u, v, h, s1), block 1 (s2, s3, t0,
 * t1), block b >= 2 the torsions t_{4b-6 ..}; uniforms are (x >> 8) 2^-24; h = h_lo +
 * (h_hi - h_lo) U; the quaternion follows Shoemake's method from (s1, s2, s3); phi_k = 2 pi t_k.
 * n_tors <= 16.  d_raw (nullable) receives the raw 32-bit outputs [n][blocks][4]. */
gff_status gff_propose_uniform(int n_rep, int n_tors, uint64_t seed, uint32_t round, float h_lo, float h_hi,
                               float *d_dof, uint32_t *d_raw, void *stream);

/* Continuous-flow relaxation (the batching of Section "Configuration sampling on GPU" with
 * replicas replaced as they finish): per replica r of `plan`, d_mode[r] = 1 loads a new
 * proposal -- positions from d_pos_src [3][N] (same layout as state->d_pos), velocities 0,
 * FIRE dt = dt0, alpha = alpha0, positive-power count 0 (FIRE arrays nullable), status 0;
 * d_mode[r] = 2 freezes the replica (velocities 0, status GFF_REP_CONVERGED: later launches
 * evaluate it without moving it); 0 leaves it.  Relaxing in launches of a fixed step count
 * with refills in between gives each proposal the trajectory of one uninterrupted launch.
 * d_pos_src may be state->d_pos itself (mode 1 then only resets velocities and FIRE state).
 * All buffers are caller-owned device memory; asynchronous on `stream`. */
gff_status gff_refill(const gff_plan *plan, const int *d_mode, const float *d_pos_src, float dt0, float alpha0,
                      const gff_state *state, void *stream);

/* Pose construction from DOF (rows of dof_stride floats) for every replica of `plan`:
 * reference geometry of the type; each rotatable torsion k in order set to phi_k by rotating
 * its moving atoms about the j->k bond; rotation about the centroid by the quaternion;
 * translation of the centroid to (u Lx, v Ly) and of the lowest atom to z_top + h.
 * Writes d_pos [3][N]. */
gff_status gff_pose_from_dof(const gff_topology *topo, const gff_plan *plan, const float *d_dof, int dof_stride,
                             float Lx, float Ly, float z_top, float *d_pos, void *stream);

/* Inverse map for training the proposer: pose -> encoding [n][41] = (cos 2 pi u, sin 2 pi u,
 * cos 2 pi v, sin 2 pi v, h, quaternion with w >= 0, (cos phi_k, sin phi_k) for k < 16, zero past
 * the type's torsions).  The orientation is the rigid rotation that best maps the reference
 * geometry (with the measured torsions) onto the pose (Horn's quaternion method).
 * d_work: 3N floats of scratch. */
gff_status gff_encode_pose(const gff_topology *topo, const gff_plan *plan, const float *d_pos, float Lx, float Ly,
                           float z_top, float *d_work, float *d_enc, void *stream);

/* Encoding [n][41] -> DOF [n][7 + n_tors]: angles from the (cos, sin) pairs, quaternion
 * normalised, height clamped to [h_lo, h_hi]. */
gff_status gff_decode_dof(int n, const float *d_enc, int n_tors, float h_lo, float h_hi, float *d_dof, void *stream);

/* Distinct minima in discovery order (energy criterion): candidate c (skipped if d_ok[c] == 0;
 * d_ok nullable) is new when its energy differs by more than tol from every archived minimum
 * of the same type, including candidates accepted earlier in the batch.  New minima are
 * appended to the archive (d_arch_E, d_arch_type, count *d_arch_n, at most `capacity`);
 * d_is_new[c] = 1 for them.  Sequential in c by definition: three kernels (candidates
 * against the prior archive, candidates against each other, then one workgroup in order
 * over those that an earlier candidate lies within tol of). */
gff_status gff_dedupe_energy(int n_new, const double *d_E, const int *d_type, const int *d_ok, double tol,
                             int capacity, double *d_arch_E, int *d_arch_type, int *d_arch_n, int *d_is_new,
                             void *stream);

/* Distinct minima in discovery order (RMSD criterion, Section "Configuration sampling on
 * GPU"): two minima of one molecule type are the same when
 *   min over lattice vectors t = (a Lx, b Ly), a, b integers, of sqrt((1/n) sum_i |x_i - y_i - t|^2) <= tol,
 * atoms compared in the type's order (adsorption site and orientation count; no rotation fit,
 * no permutation); the minimising t is the lattice vector nearest the mean difference.  The
 * candidates are the plan's replicas, positions d_pos [3][N] in the plan's layout, skipped
 * where d_ok[r] == 0 (d_ok nullable) or a coordinate is non-finite; in replica order, r is
 * new when it matches no archived minimum of its type, including those accepted earlier in
 * the call, and the archive has room.  The decision is taken in FP64.
 * Archive (caller-owned, device): entry k holds atoms d_arch_pos [k][max_atoms][3] (FP32),
 * centroid d_arch_cen [k][3] (FP64, the mean of its atoms in order), type d_arch_type [k];
 * *d_arch_n (device int) entries are in use, new minima are appended up to `capacity`.
 * d_is_new [n_rep] receives 1 for the new minima.  max_atoms must cover every type in the
 * plan (<= 128).  d_work: gff_dedupe_rmsd_workspace_bytes(n_rep) bytes of device scratch.
 * Four kernels: every candidate against the prior archive, every candidate against the
 * earlier candidates, one workgroup over the candidates in order (comparing only those that
 * match an earlier candidate), and the appends and flags. */
size_t gff_dedupe_rmsd_workspace_bytes(int n_rep);
gff_status gff_dedupe_rmsd(const gff_plan *plan, const float *d_pos, const int *d_ok, float tol, float Lx, float Ly,
                           int capacity, int max_atoms, float *d_arch_pos, double *d_arch_cen, int *d_arch_type,
                           int *d_arch_n, int *d_is_new, void *d_work, size_t work_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * sampling loops, harnesses that forbid allocation): gff_dedupe_rmsd with its scratch in a
 * static device array of GFF_DEDUPE_NOALLOC_MAX_REP candidates (2.25 MiB per GPU, held
 * until the process ends) instead of a workspace argument.  Same arguments, results and
 * errors as gff_dedupe_rmsd; plans of more than GFF_DEDUPE_NOALLOC_MAX_REP replicas return
 * GFF_EWORKSPACE and enqueue nothing.  Calls no allocating routine; the scratch address of a
 * device is looked up on the first call made with that device current.  All calls on one
 * GPU share the array: calls that overlap in time on one GPU (different streams, or other
 * host threads) race and give undefined results; calls in one stream are ordered. */
#define GFF_DEDUPE_NOALLOC_MAX_REP 65536
gff_status gff_dedupe_rmsd_noalloc(const gff_plan *plan, const float *d_pos, const int *d_ok, float tol, float Lx,
                                   float Ly, int capacity, int max_atoms, float *d_arch_pos, double *d_arch_cen,
                                   int *d_arch_type, int *d_arch_n, int *d_is_new, void *stream);

/* ------------------------------------------------------------------ learned proposer */

/* A 4-layer MLP (widths 96 -> 256 -> 256 -> 256 -> 41, SiLU between layers) maps
 * [64 standard-normal noise values | 32-d embedding of the molecule type] to the pose
 * encoding of gff_encode_pose.  Weights are FP32 masters with BF16 copies; every GEMM runs
 * on BF16 MFMA with FP32 accumulation.  Parameter layout (FP32): W1 [256][96], b1 [256],
 * W2 [256][256], b2, W3 [256][256], b3, W4 [41][256], b4 [41], embedding [n_types][32].
 * The proposer is trained on the distinct minima the relaxation finds (IMLE, Li & Malik 2018):
 * for every minimum K noise draws are decoded, the nearest output is kept, and a step on the
 * masked squared error (quaternion compared up to sign) follows. */
typedef struct gff_mlp_s gff_mlp;
size_t gff_mlp_n_params(int n_types);
/* copies params_h (FP32, gff_mlp_n_params floats) to the device; Adam moments start at 0 */
gff_status gff_mlp_create(int n_types, const float *params_h, gff_mlp **out);
void gff_mlp_destroy(gff_mlp *mlp);
/* synchronous copies of the FP32 parameters and/or the last gradient (either may be NULL) */
gff_status gff_mlp_get_params(const gff_mlp *mlp, float *params_h, float *grads_h);
/* Bytes of the device workspace (caller-owned, overwritten) that gff_mlp_forward and
 * gff_mlp_train_step need for `batch` rows: activations, pre-activations, gradients and the
 * split-K partial sums of the weight gradients.  Calls sharing one workspace must not overlap. */
size_t gff_mlp_workspace_bytes(int batch);
/* d_noise [batch][64], d_type [batch] -> d_out [batch][41]; GFF_EWORKSPACE if work_bytes is
 * below gff_mlp_workspace_bytes(batch) */
gff_status gff_mlp_forward(gff_mlp *mlp, int batch, const float *d_noise, const int *d_type, float *d_out,
                           void *d_work, size_t work_bytes, void *stream);
/* one training step on (noise, type, target encoding, torsion count) rows: outputs, per-sample
 * loss (nullable), gradient of the batch mean into the model, then Adam with step lr (lr <= 0:
 * gradient only) */
gff_status gff_mlp_train_step(gff_mlp *mlp, int batch, const float *d_noise, const int *d_type,
                              const float *d_target, const int *d_ntors, float lr, float *d_out, float *d_loss,
                              void *d_work, size_t work_bytes, void *stream);
/* IMLE selection: d_cand_out [n][K][41] against d_target [n][41]: index of the nearest
 * candidate per row (ties: lowest index) and its distance (nullable) */
gff_status gff_imle_select(int n, int K, const float *d_cand_out, const float *d_target, const int *d_ntors,
                           int *d_best, float *d_best_dist, void *stream);
/* n standard normals by Box-Muller from Philox4x32-10: counter (q, round, 1, q >> 32) with
 * q = i/4 gives outputs 4q..4q+3; uniforms ((x >> 8) + 0.5) 2^-24; pairs (u0,u1), (u2,u3) */
gff_status gff_normal_philox(long n, uint64_t seed, uint32_t round, float *d_out, void *stream);
/* dst[r][:] = src[r K + idx[r]][:] for rows of `len` floats (idx clamped to [0, K)): picks the
 * IMLE-selected noise rows */
gff_status gff_gather_rows(int n, int len, const float *d_src, int K, const int *d_idx, float *d_dst, void *stream);
/* C [M][N] (FP32) = A [M][K] B [K][N] (BF16, row-major) on the MFMA tile used by the MLP */
gff_status gff_gemm_bf16(int M, int N, int K, const void *d_A, const void *d_B, float *d_C, void *stream);
/* The same tile with element strides: C[m*ldc + n] = sum_k A[m*sam + k*sak] B[k*sbk + n*sbn]
 * (BF16 inputs as raw 16-bit words, FP32 output; strides >= 1, ldc >= N).  Operands
 * contiguous along k or along their row index are read with 16-byte loads when 16-byte
 * aligned.  With d_work (at least gff_gemm_bf16_workspace_bytes(), device memory owned by the
 * caller, overwritten) a product of fewer than 64 output tiles of 64 x 64 and K >= 128 splits
 * K over blocks, the FP32 partial sums added in slice order by a second kernel; d_work NULL:
 * one pass over K.  Results are deterministic either way.  GFF_EWORKSPACE when work_bytes is
 * too small; asynchronous on `stream`. */
size_t gff_gemm_bf16_workspace_bytes(void);
gff_status gff_gemm_bf16_strided(int M, int N, int K, const void *d_A, long sam, long sak, const void *d_B,
                                 long sbk, long sbn, float *d_C, long ldc, void *d_work, size_t work_bytes,
                                 void *stream);

/* ------------------------------------------------------------------ measurement aid */

/* Random-gather bandwidth probe (not a step of the method: the peak against which the
 * replica kernel's interpolation traffic is compared).  n_threads (a multiple of 256) lanes
 * in quads; quad q draws `iters` chunk indices c from xorshift32 (h ^= h << 13; h ^= h >> 17;
 * h ^= h << 5) started at h = q * 0x9E3779B9 ^ seed (0x6D2B79F5 if that is 0), c = the high
 * 32 bits of h * (bytes / 64); lane s of the quad loads the 16-byte word s of 64-byte chunk c
 * of d_buf.  d_sink[n_threads] receives each lane's XOR of the 32-bit words it loaded.
 * d_buf: device, 16-byte aligned, `bytes` a multiple of 64 (at most 2^32 chunks).  Bytes moved
 * per call: n_threads * iters * 16.  Asynchronous on `stream`; GFF_EINVAL on bad arguments. */
gff_status gff_gather_probe(const void *d_buf, size_t bytes, int n_threads, int iters, unsigned seed,
                            unsigned *d_sink, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* GRIDFF_H */
