// Internal types of libgridff: device tables of molecule types and work lists.
// Not part of the public ABI (see include/gridff.h).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <vector>
#include <cstdint>
#include "gridff.h"

namespace gff {

constexpr int kMaxAtoms = 128;             // atoms per molecule type (4 x 32-bit exclusion words)

// Evaluation layout of a B-spline grid along z: a column's padded planes p = 0 .. nz+2
// (plane p holds node p-1) are stored as overlapping blocks of kZBlock nodes, block b
// holding planes kZStep b .. kZStep b + kZBlock - 1.  The four planes k .. k+3 that an
// interpolation in cell k reads all lie in block k / kZStep, so with a block of 8 nodes
// (128 bytes F32, 64 bytes F16, aligned to that size) every column window is one L2 line
// instead of straddling two for three cells in eight; the cost is 8/5 of the plain column.
constexpr int kZBlock = 8, kZStep = 5;
__host__ __device__ constexpr int col_nodes(int nz) { return ((nz - 1) / kZStep + 1) * kZBlock; }
// position in the column of padded plane k (k = 0 .. nz-1), the window's first node
__host__ __device__ constexpr int window_node(int k) { return k + (kZBlock - kZStep) * (int)((unsigned)k / kZStep); }

constexpr float kEvPerAmuA2Fs2 = 103.6426965268f;  // 1 amu A^2 / fs^2 in eV
constexpr double kDefaultKe = 14.3996454784;

// Philox4x32 with 10 rounds (Salmon, Moraes, Dror & Shaw, SC'11), counter c in place, key
// (k0, k1) bumped by the Weyl constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
}

// Three standard normals from one Philox block by the Box-Muller transform, with the
// uniforms u = ((x >> 9) + 1/2) 2^-23 (exact in FP32, strictly inside (0, 1)).
__device__ __forceinline__ float3 philox_normal3(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1) {
    uint32_t c[4] = {c0, c1, c2, c3};
    philox4x32_10(c, k0, k1);
    float u[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) u[k] = ((float)(c[k] >> 9) + 0.5f) * (1.f / 8388608.f);
    const float r0 = sqrtf(-2.f * logf(u[0])), r2 = sqrtf(-2.f * logf(u[2]));
    float s1, co1;
    sincospif(2.f * u[1], &s1, &co1);
    return make_float3(r0 * co1, r0 * s1, r2 * cospif(2.f * u[3]));
}

struct TypeInfo {              // per molecule type
    int n;                     // atoms
    int abase;                 // first entry in the per-type-atom arrays
    int tbase;                 // first torsion of the type in the torsion-term table
    int nt;                    // torsion terms of the type
    // the type's torsion topology as one block of 16-byte words, copied to LDS by the replica
    // kernel: [incT: n int2 (first incidence, count), padded to (n + 1) / 2 words][incG: n + 1
    // int4][torsion terms, one word each][torsion incidences, int (term << 2 | slot),
    // padded].  An atom's incidences are stored grouped by its slot in the term (i, j, k, l),
    // terms ascending within a group; incG[a] = (first incidence, ends of the slot-0, slot-1
    // and slot-2 groups), the slot-3 group ending at incG[a + 1].x.  Indices inside are
    // relative to the block's own sections
    int blob_off, blob_words;  // first word in the blob table, length in words
    int o_tor, o_tinc;         // section starts (words); incT at word 0, incG at (n + 1) / 2
};

// Torsion term: atoms (i,j,k,l) packed seven bits each with the multiplicity n in the top
// four bits, barrier V and (cos phi0, sin phi0).
struct TorDef { int ijkln; float V, c0, s0; };

// One entry per (atom, incident term).  `slot` is the atom's position in the term; the
// slot-0 entry carries the term's energy so every term is counted once.
struct BondInc { int other; int slot; float k; float r0; };
struct AngInc  { int abcs; float k, cos0, pad; };   // a | b << 8 | c << 16 | slot << 24, b = vertex

struct DevTopo {
    const TypeInfo *types;
    const float4 *plqm;        // [type atoms] P, L, Q, 1/(m * 103.6427)
    const float *khalf;        // [type atoms] m * 103.6427 / 2
    const uint4 *excl;         // [type atoms] bit j: pair excluded (self, 1-2, 1-3)
    const float4 *refpos;      // [type atoms] reference geometry (pose construction)
    const int4 *rotq;          // [rotatable torsions of all types] quad
    const uint4 *rotm;         // [same] 128-bit moving mask
    const int2 *rotinfo;       // [types] first rotatable torsion, count
    const int4 *incA;          // [type atoms] bond start, bond count, angle start, angle count
    const BondInc *bnd;        // one per (atom, incident bond)
    const AngInc *ang;         // one per (atom, incident angle)
    // per-type torsion blocks (TypeInfo::blob_off): per atom (incidence start, count); TorDef
    // terms; torsion incidences (term << 2 | slot)
    const int4 *blob;
};

}  // namespace gff

struct gff_topology_s {
    int n_types;
    std::vector<int> ntors;
    std::vector<int> blob_words;   // per type: LDS words of its torsion block
    float alpha, ke;
    std::vector<int> natoms;
    std::vector<int> nrot;
    gff::DevTopo dev;
    std::vector<void *> allocations;
};

struct gff_plan_s {
    int n_rep, n_atoms, n_packs;
    int block_threads, grid_blocks, max_n;
    int lanes_per_atom;        // 1, 2 or 4 (B-spline relaxation and dynamics launches)
    int lds_limit;             // the device's LDS bytes per block
    int tres_max;              // largest (replicas per pack) x (torsion terms) of the batch
    int max_pack_reps;         // largest number of replicas in one pack
    int topo_words;            // largest torsion block of the batch (16-byte words)
    int4 *d_packs;             // type, replicas in pack, first entry in d_pack_reps, pad
    int *d_pack_reps;          // replica ids in pack order
    int *d_atom_off;           // [n_rep+1]
    int *d_rep_type;           // [n_rep]
    std::vector<int> atom_off_h;
    std::vector<int> rep_type_h;
};

namespace gff {
inline gff_status hip_status(hipError_t e) { return e == hipSuccess ? GFF_OK : GFF_EHIP; }
}

// Dynamic LDS of the replica kernel: five float4 slots and one int per atom slot (lanes / lanes
// per atom), two float4 per
// (replica, torsion term), six doubles of NVE drift record per replica, three flag words (16 bytes) and
// the largest torsion block of the batch.
inline size_t replica_lds_bytes(int slots, int tres_max, int max_pack_reps, int topo_words) {
    return (size_t)slots * (5 * 16 + 4) + (size_t)tres_max * 32 + (size_t)max_pack_reps * 48 + 16 +
           (size_t)topo_words * 16;
}

// All-atom comparison mode: substrate atoms with their Pauli/London factors on the device.
struct gff_direct_s {
    int n, nimg;
    float alpha, Lx, Ly;
    float4 *d_xyza;            // x, y, z, eps e^{2 alpha R}
    float2 *d_bq;              // eps e^{alpha R}, q
    std::vector<void *> allocations;
};

