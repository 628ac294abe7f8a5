// Host side of libgridff: molecule-type tables, replica work lists, status strings.
#include "gff_internal.hpp"
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

using namespace gff;

extern "C" const char *gff_status_string(int s) {
    switch (s) {
        case GFF_OK: return "ok";
        case GFF_EINVAL: return "invalid argument";
        case GFF_EUNSUPPORTED: return "unsupported request";
        case GFF_EHIP: return "HIP runtime or launch error";
        case GFF_EWORKSPACE: return "workspace too small";
        case GFF_ENOMEM: return "device allocation failed";
        default: return "unknown status";
    }
}

namespace {

template <class T>
gff_status upload(std::vector<void *> &owned, const std::vector<T> &h, const T **out) {
    size_t bytes = std::max<size_t>(1, h.size()) * sizeof(T);
    void *d = nullptr;
    if (hipMalloc(&d, bytes) != hipSuccess) return GFF_ENOMEM;
    owned.push_back(d);
    if (!h.empty() && hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return GFF_EHIP;
    *out = static_cast<const T *>(d);
    return GFF_OK;
}

void free_all(std::vector<void *> &owned) {
    for (void *p : owned) (void)hipFree(p);
    owned.clear();
}

bool valid_type(const gff_mol_type &m) {
    if (m.n_atoms < 1 || m.n_atoms > kMaxAtoms) return false;
    if (!m.eps || !m.R || !m.q || !m.mass) return false;
    auto in = [&](int i) { return i >= 0 && i < m.n_atoms; };
    if (m.n_bonds < 0 || (m.n_bonds > 0 && (!m.bonds || !m.bond_k || !m.bond_r0))) return false;
    for (int b = 0; b < m.n_bonds; ++b)
        if (!in(m.bonds[2 * b]) || !in(m.bonds[2 * b + 1]) || m.bonds[2 * b] == m.bonds[2 * b + 1]) return false;
    if (m.n_angles < 0 || (m.n_angles > 0 && (!m.angles || !m.angle_k || !m.angle_cos0))) return false;
    for (int a = 0; a < 3 * m.n_angles; ++a) if (!in(m.angles[a])) return false;
    if (m.n_tors < 0 || (m.n_tors > 0 && (!m.tors || !m.tors_V || !m.tors_n || !m.tors_phi0))) return false;
    for (int t = 0; t < 4 * m.n_tors; ++t) if (!in(m.tors[t])) return false;
    for (int t = 0; t < m.n_tors; ++t) if (m.tors_n[t] < 1 || m.tors_n[t] > 12) return false;
    if (m.n_rot < 0 || (m.n_rot > 0 && (!m.rot_quads || !m.rot_mask))) return false;
    for (int t = 0; t < 4 * m.n_rot; ++t) if (!in(m.rot_quads[t])) return false;
    for (int a = 0; a < m.n_atoms; ++a)
        if (!(m.mass[a] > 0.f) || !std::isfinite(m.eps[a]) || !std::isfinite(m.R[a]) || !std::isfinite(m.q[a]))
            return false;
    return true;
}

}  // namespace

extern "C" gff_status gff_topology_create(const gff_mol_type *types, int n_types, float alpha, float k_e,
                                          gff_topology **out) {
    if (!types || n_types < 1 || !out || !(alpha > 0.f)) return GFF_EINVAL;
    for (int t = 0; t < n_types; ++t) if (!valid_type(types[t])) return GFF_EINVAL;
    auto *T = new gff_topology_s();
    T->n_types = n_types;
    T->alpha = alpha;
    T->ke = k_e > 0.f ? k_e : (float)kDefaultKe;
    std::vector<TypeInfo> ti(n_types);
    std::vector<float4> plqm, refpos;
    std::vector<float> khalf;
    std::vector<uint4> excl;
    std::vector<int4> incA, rotq;
    std::vector<int4> incT;
    std::vector<int2> rotinfo(n_types);
    std::vector<BondInc> bnd;
    std::vector<AngInc> ang;
    std::vector<TorDef> tdef;
    std::vector<int> tinc;
    std::vector<uint4> rotm;
    std::vector<int4> blob;
    for (int t = 0; t < n_types; ++t) {
        const gff_mol_type &m = types[t];
        const int n = m.n_atoms;
        ti[t] = TypeInfo{n, (int)plqm.size(), (int)tdef.size(), m.n_tors, 0, 0, 0, 0};
        const int tinc0 = (int)tinc.size();
        T->natoms.push_back(n);
        T->ntors.push_back(m.n_tors);
        for (int q = 0; q < m.n_tors; ++q) {
            const int *Q4 = m.tors + 4 * q;
            const double ph = m.tors_phi0[q];
            tdef.push_back(TorDef{Q4[0] | (Q4[1] << 7) | (Q4[2] << 14) | (Q4[3] << 21) | (m.tors_n[q] << 28),
                                  m.tors_V[q], (float)std::cos(ph), (float)std::sin(ph)});
        }
        T->nrot.push_back(m.n_rot);
        // adjacency and exclusions (self, 1-2, 1-3)
        std::vector<std::vector<char>> adj(n, std::vector<char>(n, 0));
        for (int b = 0; b < m.n_bonds; ++b) {
            int i = m.bonds[2 * b], j = m.bonds[2 * b + 1];
            adj[i][j] = adj[j][i] = 1;
        }
        for (int a = 0; a < n; ++a) {
            const double eps = m.eps[a], R = m.R[a];
            const double P = eps * std::exp(2.0 * alpha * R), L = -2.0 * eps * std::exp(alpha * R);
            const double macc = (double)m.mass[a] * kEvPerAmuA2Fs2;
            plqm.push_back(make_float4((float)P, (float)L, m.q[a], (float)(1.0 / macc)));
            khalf.push_back((float)(0.5 * macc));
            unsigned w[4] = {0, 0, 0, 0};
            for (int b = 0; b < n; ++b) {
                bool e = (a == b) || adj[a][b];
                for (int c = 0; c < n && !e; ++c) if (adj[a][c] && adj[c][b]) e = true;
                if (e) w[b >> 5] |= 1u << (b & 31);
            }
            excl.push_back(make_uint4(w[0], w[1], w[2], w[3]));
            const float *rp = m.ref_pos;
            refpos.push_back(rp ? make_float4(rp[3 * a], rp[3 * a + 1], rp[3 * a + 2], 0.f) : make_float4(0, 0, 0, 0));
            // incident terms
            int4 ia;
            ia.x = (int)bnd.size();
            for (int b = 0; b < m.n_bonds; ++b) {
                int i = m.bonds[2 * b], j = m.bonds[2 * b + 1];
                if (i == a) bnd.push_back(BondInc{j, 0, m.bond_k[b], m.bond_r0[b]});
                else if (j == a) bnd.push_back(BondInc{i, 1, m.bond_k[b], m.bond_r0[b]});
            }
            ia.y = (int)bnd.size() - ia.x;
            ia.z = (int)ang.size();
            for (int q = 0; q < m.n_angles; ++q) {
                const int *A3 = m.angles + 3 * q;
                for (int s = 0; s < 3; ++s)
                    if (A3[s] == a) {
                        ang.push_back(AngInc{A3[0] | (A3[1] << 8) | (A3[2] << 16) | (s << 24), m.angle_k[q],
                                             m.angle_cos0[q], 0.f});
                        break;
                    }
            }
            ia.w = (int)ang.size() - ia.z;
            incA.push_back(ia);
            // incident torsion terms grouped by the atom's slot (i, j, k, l), terms ascending
            // within a slot: (first entry, end of the slot-0, slot-1 and slot-2 groups)
            int ends[4];
            const int first = (int)tinc.size();
            for (int s = 0; s < 4; ++s) {
                for (int q = 0; q < m.n_tors; ++q) {
                    const int *Q4 = m.tors + 4 * q;
                    int slot = -1;
                    for (int u = 0; u < 4 && slot < 0; ++u) if (Q4[u] == a) slot = u;
                    if (slot == s) tinc.push_back((q << 2) | s);
                }
                ends[s] = (int)tinc.size();
            }
            incT.push_back(make_int4(first, ends[0], ends[1], ends[2]));
        }
        // the type's torsion block (indices relative to its own sections)
        {
            TypeInfo &T0 = ti[t];
            std::vector<int4> b;
            auto words = [](size_t bytes) { return (int)((bytes + 15) / 16); };
            const int tend = (int)tinc.size() - tinc0;          // where the last atom's slot-3 group ends
            std::vector<int> it2;
            for (int a = 0; a < n; ++a) {
                const int first = incT[T0.abase + a].x - tinc0;
                const int end = a + 1 < n ? incT[T0.abase + a + 1].x - tinc0 : tend;
                it2.push_back(first); it2.push_back(end - first);
            }
            it2.resize((size_t)words(it2.size() * 4) * 4, 0);
            for (size_t k = 0; k < it2.size(); k += 4) b.push_back(make_int4(it2[k], it2[k + 1], it2[k + 2], it2[k + 3]));
            // incG starts at word ceil(8 n / 16) = (n + 1) / 2, where the kernel looks for it
            for (int a = 0; a < n; ++a) {
                const int4 r = incT[T0.abase + a];
                b.push_back(make_int4(r.x - tinc0, r.y - tinc0, r.z - tinc0, r.w - tinc0));
            }
            b.push_back(make_int4(tend, tend, tend, tend));
            T0.o_tor = (int)b.size();
            for (int q = 0; q < m.n_tors; ++q) {
                int4 w; std::memcpy(&w, &tdef[T0.tbase + q], 16); b.push_back(w);
            }
            T0.o_tinc = (int)b.size();
            std::vector<int> tc(tinc.begin() + tinc0, tinc.end());
            tc.resize((size_t)words(tc.size() * 4) * 4, 0);
            for (size_t k = 0; k < tc.size(); k += 4) b.push_back(make_int4(tc[k], tc[k + 1], tc[k + 2], tc[k + 3]));
            T0.blob_off = (int)blob.size();
            T0.blob_words = (int)b.size();
            blob.insert(blob.end(), b.begin(), b.end());
            T->blob_words.push_back(T0.blob_words);
        }
        rotinfo[t] = make_int2((int)rotq.size(), m.n_rot);
        for (int k = 0; k < m.n_rot; ++k) {
            const int *q = m.rot_quads + 4 * k;
            rotq.push_back(make_int4(q[0], q[1], q[2], q[3]));
            unsigned w[4] = {0, 0, 0, 0};
            for (int a = 0; a < n; ++a) if (m.rot_mask[(size_t)k * n + a]) w[a >> 5] |= 1u << (a & 31);
            rotm.push_back(make_uint4(w[0], w[1], w[2], w[3]));
        }
    }
    gff_status rc = GFF_OK;
    auto &o = T->allocations;
    DevTopo &d = T->dev;
    if ((rc = upload(o, ti, &d.types)) || (rc = upload(o, plqm, &d.plqm)) || (rc = upload(o, khalf, &d.khalf)) ||
        (rc = upload(o, excl, &d.excl)) || (rc = upload(o, incA, &d.incA)) || (rc = upload(o, bnd, &d.bnd)) ||
        (rc = upload(o, ang, &d.ang)) || (rc = upload(o, blob, &d.blob)) ||
        (rc = upload(o, refpos, &d.refpos)) || (rc = upload(o, rotq, &d.rotq)) || (rc = upload(o, rotm, &d.rotm)) ||
        (rc = upload(o, rotinfo, &d.rotinfo))) {
        free_all(o);
        delete T;
        return rc;
    }
    *out = T;
    return GFF_OK;
}

extern "C" void gff_topology_destroy(gff_topology *T) {
    if (!T) return;
    free_all(T->allocations);
    delete T;
}

extern "C" gff_status gff_plan_create(const gff_topology *topo, int n_rep, const int *rep_type_h,
                                      const gff_launch *launch, gff_plan **out) {
    if (!topo || n_rep < 0 || (n_rep > 0 && !rep_type_h) || !out) return GFF_EINVAL;
    int BT = 256, rpb_cap = 0, grid = 0, lpa = 1;
    if (launch) {
        BT = launch->block_threads > 0 ? launch->block_threads : 256;
        rpb_cap = launch->reps_per_block;
        grid = launch->grid_blocks;
        lpa = launch->lanes_per_atom > 0 ? launch->lanes_per_atom : 1;
    }
    if (BT % 64 != 0 || BT < 64 || BT > 1024) return GFF_EINVAL;
    if (lpa != 1 && lpa != 2 && lpa != 4) return GFF_EINVAL;
    const int NS = BT / lpa;                              // atom slots per block
    std::vector<int> atom_off(n_rep + 1, 0);
    int max_n = 0;
    for (int r = 0; r < n_rep; ++r) {
        const int t = rep_type_h[r];
        if (t < 0 || t >= topo->n_types) return GFF_EINVAL;
        atom_off[r + 1] = atom_off[r] + topo->natoms[t];
        max_n = std::max(max_n, topo->natoms[t]);
    }
    if (max_n > NS) return GFF_EUNSUPPORTED;
    // packs of same-type replicas, densest packing of one lane per atom
    std::vector<std::vector<int>> by_type(topo->n_types);
    for (int r = 0; r < n_rep; ++r) by_type[rep_type_h[r]].push_back(r);
    std::vector<int> order(topo->n_types);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return topo->natoms[a] > topo->natoms[b]; });
    // LDS per block: 84 bytes per atom slot, the largest torsion block, 48 bytes per replica and
    // 32 bytes per (replica, torsion term); packs of torsion-heavy types hold fewer replicas
    // when the block's LDS would overflow
    int dev = 0, lds_limit = 65536;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
            lds_limit = v;
    }
    int topo_words = 0;                                   // largest torsion block of the batch
    for (int t = 0; t < topo->n_types; ++t)
        if (!by_type[t].empty()) topo_words = std::max(topo_words, topo->blob_words[t]);
    const long lane_lds = (long)NS * (5 * 16 + 4) + 16 + 16L * topo_words;
    if (lane_lds >= lds_limit) return GFF_EUNSUPPORTED;
    std::vector<int4> packs;
    std::vector<int> reps;
    int tres_max = 0, max_pack_reps = 0;
    for (int t : order) {
        const int n = topo->natoms[t];
        int rpb = NS / n;
        if (rpb_cap > 0) rpb = std::min(rpb, rpb_cap);
        if (topo->ntors[t] > 0 && !by_type[t].empty()) {
            const long fit = (lds_limit - lane_lds - 48L * rpb) / (32L * topo->ntors[t]);
            if (fit < 1) return GFF_EUNSUPPORTED;
            rpb = (int)std::min<long>(rpb, fit);
        }
        const auto &L = by_type[t];
        if (!L.empty()) tres_max = std::max(tres_max, (int)std::min<size_t>(rpb, L.size()) * topo->ntors[t]);
        for (size_t s = 0; s < L.size(); s += rpb) {
            const int cnt = (int)std::min<size_t>(rpb, L.size() - s);
            packs.push_back(make_int4(t, cnt, (int)reps.size(), 0));
            max_pack_reps = std::max(max_pack_reps, cnt);
            for (int k = 0; k < cnt; ++k) reps.push_back(L[s + k]);
        }
    }
    auto *P = new gff_plan_s();
    P->n_rep = n_rep; P->n_atoms = atom_off[n_rep]; P->n_packs = (int)packs.size();
    P->block_threads = BT; P->grid_blocks = grid; P->max_n = max_n; P->tres_max = tres_max;
    P->max_pack_reps = max_pack_reps; P->topo_words = topo_words;
    P->lanes_per_atom = lpa; P->lds_limit = lds_limit;
    if ((long)replica_lds_bytes(NS, tres_max, max_pack_reps, topo_words) > lds_limit) {
        delete P;
        return GFF_EUNSUPPORTED;
    }
    P->atom_off_h = atom_off;
    P->rep_type_h.assign(rep_type_h, rep_type_h + n_rep);
    std::vector<void *> owned;
    const int4 *dp; const int *dr, *da, *dt;
    gff_status rc;
    if ((rc = upload(owned, packs, &dp)) || (rc = upload(owned, reps, &dr)) || (rc = upload(owned, atom_off, &da)) ||
        (rc = upload(owned, P->rep_type_h, &dt))) {
        free_all(owned);
        delete P;
        return rc;
    }
    P->d_packs = const_cast<int4 *>(dp);
    P->d_pack_reps = const_cast<int *>(dr);
    P->d_atom_off = const_cast<int *>(da);
    P->d_rep_type = const_cast<int *>(dt);
    *out = P;
    return GFF_OK;
}

extern "C" void gff_plan_destroy(gff_plan *P) {
    if (!P) return;
    (void)hipFree(P->d_packs);
    (void)hipFree(P->d_pack_reps);
    (void)hipFree(P->d_atom_off);
    (void)hipFree(P->d_rep_type);
    delete P;
}

extern "C" int gff_plan_n_atoms(const gff_plan *P) { return P ? P->n_atoms : -1; }
extern "C" int gff_plan_n_packs(const gff_plan *P) { return P ? P->n_packs : -1; }

extern "C" gff_status gff_plan_atom_offsets(const gff_plan *P, int *atom_off_h) {
    if (!P || !atom_off_h) return GFF_EINVAL;
    std::memcpy(atom_off_h, P->atom_off_h.data(), sizeof(int) * P->atom_off_h.size());
    return GFF_OK;
}
