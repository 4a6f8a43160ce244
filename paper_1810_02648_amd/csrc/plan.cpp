// Template creation: topology tables and the tiled execution plan (host code).
//
// The matrix-free J^T J p of the non-rigid stage (Sec. 4, non-rigid paragraph)
// touches, per vertex, its 4 bound nodes.  The plan groups vertices by their
// nearest node, orders nodes breadth-first over the node graph and cuts the
// resulting vertex sequence into tiles of at most 256 vertices.  Each tile
// accumulates the 6-vectors of the nodes it touches ("slots") in LDS and
// writes one partial per slot; a per-node list of partials, in tile order,
// makes the final sum deterministic without atomics.  Every node's outgoing
// regulariser edges are handled by exactly one tile (its owner).
#include <algorithm>
#include <cstring>
#include <map>
#include <queue>
#include <vector>

#include "common.hpp"

namespace cap {

namespace {

template <typename T>
int copy_down(std::vector<T> &dst, const T *src, size_t n) {
    dst.resize(n);
    if (n) CAP_HIP(hipMemcpy(dst.data(), src, n * sizeof(T), hipMemcpyDeviceToHost));
    return CAPTURE_OK;
}

struct Blob {
    std::vector<uint8_t> bytes;
    template <typename T>
    size_t add(const std::vector<T> &v) {
        size_t off = (bytes.size() + 255) & ~size_t(255);
        bytes.resize(off + std::max<size_t>(v.size() * sizeof(T), 1));
        if (!v.empty()) std::memcpy(bytes.data() + off, v.data(), v.size() * sizeof(T));
        return off;
    }
};

// Mesh edges with their adjacent faces (edge-manifold check) and the
// vertex -> incident faces lists, ascending.
int topology(const std::vector<int> &tri, int nv, int nf, std::vector<int> &medge, int &nme,
             std::vector<int> &vf_beg, std::vector<int> &vf_face) {
    // ---- mesh edges with their adjacent faces (edge-manifold check)
    std::vector<std::pair<uint64_t, int>> ek;
    ek.reserve(size_t(3) * nf);
    for (int f = 0; f < nf; ++f)
        for (int c = 0; c < 3; ++c) {
            uint64_t a = tri[size_t(c) * nf + f], b = tri[size_t((c + 1) % 3) * nf + f];
            if (a == b) return fail(CAPTURE_EINVAL, "template: degenerate triangle");
            uint64_t lo = std::min(a, b), hi = std::max(a, b);
            ek.push_back({(lo << 32) | hi, f});
        }
    std::sort(ek.begin(), ek.end());
    std::vector<int> me[4];
    for (size_t i = 0; i < ek.size();) {
        size_t j = i;
        while (j < ek.size() && ek[j].first == ek[i].first) ++j;
        if (j - i > 2) return fail(CAPTURE_EINVAL, "template: mesh is not edge-manifold");
        me[0].push_back(int(ek[i].first >> 32));
        me[1].push_back(int(ek[i].first & 0xffffffffu));
        me[2].push_back(ek[i].second);
        me[3].push_back(j - i == 2 ? ek[i + 1].second : -1);
        i = j;
    }
    nme = int(me[0].size());
    medge.clear();
    for (int k = 0; k < 4; ++k) medge.insert(medge.end(), me[k].begin(), me[k].end());

    // ---- vertex -> incident faces, ascending
    vf_beg.assign(nv + 1, 0);
    vf_face.assign(size_t(3) * nf, 0);
    for (int f = 0; f < nf; ++f)
        for (int c = 0; c < 3; ++c) vf_beg[tri[size_t(c) * nf + f] + 1]++;
    for (int v = 0; v < nv; ++v) vf_beg[v + 1] += vf_beg[v];
    {
        std::vector<int> fill(vf_beg.begin(), vf_beg.end() - 1);
        for (int f = 0; f < nf; ++f)
            for (int c = 0; c < 3; ++c) vf_face[fill[tri[size_t(c) * nf + f]]++] = f;
    }

    return CAPTURE_OK;
}

}  // namespace

int build_template(const capture_template_desc *d, capture_template **out, int device) {
    const int nv = d->n_vertices, nf = d->n_triangles, nn = d->n_nodes;
    const int vcap = d->vertices_per_tile > 0 ? d->vertices_per_tile : kMaxTileVerts;
    if (nv < 1 || nf < 1 || nn < 4 || nn > nv || nn > 65536)
        return fail(CAPTURE_EINVAL, "template: need n_vertices >= 1, n_triangles >= 1, 4 <= n_nodes <= n_vertices, n_nodes <= 65536");
    if (vcap > kMaxTileVerts) return fail(CAPTURE_EUNSUPPORTED, "template: vertices_per_tile must be <= 256");
    if (!d->tri || !d->node_vertex || !d->bind_idx || !d->bind_w || !d->edge_dst)
        return fail(CAPTURE_EINVAL, "template: null array");
    std::vector<int> tri, nvtx, bidx, edst;
    std::vector<float> bw;
    int rc;
    if ((rc = copy_down(tri, d->tri, size_t(3) * nf))) return rc;
    if ((rc = copy_down(nvtx, d->node_vertex, size_t(nn)))) return rc;
    if ((rc = copy_down(bidx, d->bind_idx, size_t(4) * nv))) return rc;
    if ((rc = copy_down(bw, d->bind_w, size_t(4) * nv))) return rc;
    if ((rc = copy_down(edst, d->edge_dst, size_t(8) * nn))) return rc;
    for (int v : tri) if (v < 0 || v >= nv) return fail(CAPTURE_EINVAL, "template: triangle index out of range");
    for (int v : nvtx) if (v < 0 || v >= nv) return fail(CAPTURE_EINVAL, "template: node_vertex out of range");
    for (int v : bidx) if (v < 0 || v >= nn) return fail(CAPTURE_EINVAL, "template: bind_idx out of range");
    for (float w : bw) if (!(w == w) || w > 3.0e38f || w < -3.0e38f) return fail(CAPTURE_ENONFINITE, "template: non-finite binding weight");
    for (int v : edst) if (v < -1 || v >= nn) return fail(CAPTURE_EINVAL, "template: edge_dst out of range");

    std::vector<int> medge, vf_beg, vf_face;
    int nme = 0;
    if ((rc = topology(tri, nv, nf, medge, nme, vf_beg, vf_face))) return rc;

    // ---- node order: breadth-first over the undirected node graph
    std::vector<std::vector<int>> adj(nn);
    for (int e = 0; e < 8; ++e)
        for (int k = 0; k < nn; ++k) {
            int l = edst[size_t(e) * nn + k];
            if (l >= 0 && l != k) { adj[k].push_back(l); adj[l].push_back(k); }
        }
    for (auto &a : adj) { std::sort(a.begin(), a.end()); a.erase(std::unique(a.begin(), a.end()), a.end()); }
    std::vector<int> order;
    std::vector<char> seen(nn, 0);
    for (int s = 0; s < nn; ++s) {
        if (seen[s]) continue;
        std::queue<int> q;
        q.push(s);
        seen[s] = 1;
        while (!q.empty()) {
            int k = q.front(); q.pop();
            order.push_back(k);
            for (int l : adj[k]) if (!seen[l]) { seen[l] = 1; q.push(l); }
        }
    }

    // ---- vertices bucketed by their nearest node (binding slot 0)
    std::vector<std::vector<int>> bucket(nn);
    for (int v = 0; v < nv; ++v) bucket[bidx[v]].push_back(v);

    // ---- tiles
    struct Tile { std::vector<int> verts, owned; std::vector<int> slots; };
    std::vector<Tile> tiles(1);
    auto has = [](const std::vector<int> &s, int k) { return std::find(s.begin(), s.end(), k) != s.end(); };
    auto contrib = [](const Tile &t) { return 4 * int(t.verts.size()) + 16 * int(t.owned.size()); };
    auto missing = [&](const Tile &t, const int *ks, int n) {
        int m = 0;
        for (int i = 0; i < n; ++i) {
            bool dup = false;
            for (int j = 0; j < i; ++j) dup |= ks[j] == ks[i];
            if (!dup && !has(t.slots, ks[i])) ++m;
        }
        return m;
    };
    for (int k : order) {
        int need[9];
        int nneed = 0;
        need[nneed++] = k;
        for (int e = 0; e < 8; ++e) { int l = edst[size_t(e) * nn + k]; if (l >= 0) need[nneed++] = l; }
        if (contrib(tiles.back()) + 16 > kMaxTileContrib ||
            int(tiles.back().slots.size()) + missing(tiles.back(), need, nneed) > kMaxTileSlots)
            tiles.emplace_back();
        Tile &t = tiles.back();
        t.owned.push_back(k);
        for (int i = 0; i < nneed; ++i) if (!has(t.slots, need[i])) t.slots.push_back(need[i]);
        for (int v : bucket[k]) {
            int ks[4];
            for (int j = 0; j < 4; ++j) ks[j] = bidx[size_t(j) * nv + v];
            Tile *cur = &tiles.back();
            if (int(cur->verts.size()) + 1 > vcap || contrib(*cur) + 4 > kMaxTileContrib ||
                int(cur->slots.size()) + missing(*cur, ks, 4) > kMaxTileSlots) {
                tiles.emplace_back();
                cur = &tiles.back();
            }
            cur->verts.push_back(v);
            for (int j = 0; j < 4; ++j) if (!has(cur->slots, ks[j])) cur->slots.push_back(ks[j]);
        }
    }
    if (tiles.back().verts.empty() && tiles.back().owned.empty()) tiles.pop_back();
    const int nt = int(tiles.size());

    std::vector<int> plan_vid, plan_pos(nv), tile_vbeg(1, 0), tile_sbeg(1, 0), slot_node, tile_obeg(1, 0),
        owned_node, list_beg(1, 0), node_pbeg(nn + 1, 0);
    std::vector<uint32_t> plan_slot, owned_cpos_t;
    std::vector<uint16_t> plan_cpos_t;       // [nv][4] in plan order
    std::vector<uint8_t> owned_slot, owned_eslot_t;
    std::vector<uint16_t> list_idx;
    std::vector<std::vector<int>> node_parts(nn);
    int max_slots = 0, max_contrib = 0;
    for (int ti = 0; ti < nt; ++ti) {
        Tile &t = tiles[ti];
        std::sort(t.slots.begin(), t.slots.end());
        std::map<int, int> sidx;
        for (size_t s = 0; s < t.slots.size(); ++s) sidx[t.slots[s]] = int(s);
        const int ns = int(t.slots.size()), nvt = int(t.verts.size()), nc = contrib(t);
        max_slots = std::max(max_slots, ns);
        max_contrib = std::max(max_contrib, nc);
        std::vector<std::vector<int>> lists(ns);
        for (int lv = 0; lv < nvt; ++lv) {
            int v = t.verts[lv];
            plan_pos[v] = int(plan_vid.size());
            plan_vid.push_back(v);
            uint32_t packed = 0;
            for (int j = 0; j < 4; ++j) {
                int s = sidx[bidx[size_t(j) * nv + v]];
                packed |= uint32_t(s) << (8 * j);
                lists[s].push_back(lv * 4 + j);
            }
            plan_slot.push_back(packed);
        }
        for (size_t o = 0; o < t.owned.size(); ++o) {
            int k = t.owned[o];
            owned_node.push_back(k);
            owned_slot.push_back(uint8_t(sidx[k]));
            for (int e = 0; e < 8; ++e) {
                int l = edst[size_t(e) * nn + k];
                int c = 4 * nvt + int(o * 8 + e) * 2;
                owned_eslot_t.push_back(l >= 0 ? uint8_t(sidx[l]) : uint8_t(255));
                if (l >= 0) {
                    lists[sidx[k]].push_back(c);
                    lists[sidx[l]].push_back(c + 1);
                }
            }
        }
        // position of every contribution in the slot-sorted order (lists concatenated)
        std::vector<int> cpos(size_t(4) * nvt + size_t(16) * t.owned.size(), 0xffff);
        const int l0 = int(list_idx.size());
        for (int s = 0; s < ns; ++s) {
            std::sort(lists[s].begin(), lists[s].end());
            for (int c : lists[s]) {
                cpos[c] = int(list_idx.size()) - l0;
                list_idx.push_back(uint16_t(c));
            }
            list_beg.push_back(int(list_idx.size()));
            node_parts[t.slots[s]].push_back(int(slot_node.size()));
            slot_node.push_back(t.slots[s]);
        }
        for (int lv = 0; lv < nvt; ++lv)
            for (int j = 0; j < 4; ++j) plan_cpos_t.push_back(uint16_t(cpos[lv * 4 + j]));
        for (size_t o = 0; o < t.owned.size(); ++o)
            for (int e = 0; e < 8; ++e) {
                const int c = 4 * nvt + int(o * 8 + e) * 2;
                owned_cpos_t.push_back(uint32_t(cpos[c]) | (uint32_t(cpos[c + 1]) << 16));
            }
        tile_vbeg.push_back(int(plan_vid.size()));
        tile_sbeg.push_back(int(slot_node.size()));
        tile_obeg.push_back(int(owned_node.size()));
        (void)nc;
    }
    if (int(plan_vid.size()) != nv || int(owned_node.size()) != nn)
        return fail(CAPTURE_EINVAL, "template: internal plan error");
    // owned edge slots: [8][nn] in owned order
    std::vector<uint8_t> owned_eslot(size_t(8) * nn);
    for (int o = 0; o < nn; ++o)
        for (int e = 0; e < 8; ++e) owned_eslot[size_t(e) * nn + o] = owned_eslot_t[size_t(o) * 8 + e];
    // the same transposed to [4][nv] and [8][nn] for coalesced loads
    std::vector<uint16_t> plan_cpos(size_t(4) * nv);
    std::vector<uint32_t> owned_cpos(size_t(8) * nn);
    for (int q = 0; q < nv; ++q)
        for (int j = 0; j < 4; ++j) plan_cpos[size_t(j) * nv + q] = plan_cpos_t[size_t(q) * 4 + j];
    for (int o = 0; o < nn; ++o)
        for (int e = 0; e < 8; ++e) owned_cpos[size_t(e) * nn + o] = owned_cpos_t[size_t(o) * 8 + e];
    std::vector<int> node_pidx, slot_dest(slot_node.size());
    for (int k = 0; k < nn; ++k) {
        for (int p : node_parts[k]) {
            slot_dest[p] = int(node_pidx.size());
            node_pidx.push_back(p);
        }
        node_pbeg[k + 1] = int(node_pidx.size());
    }
    // per slot: its node's partial range, and (bit 31 of the end) whether the
    // slot's tile owns the node (each node is owned by exactly one tile)
    std::vector<int> slot_pb(slot_node.size()), slot_pe(slot_node.size());
    for (size_t p = 0; p < slot_node.size(); ++p) {
        slot_pb[p] = node_pbeg[slot_node[p]];
        slot_pe[p] = node_pbeg[slot_node[p] + 1];
    }
    for (int ti = 0; ti < nt; ++ti)
        for (int o = tile_obeg[ti]; o < tile_obeg[ti + 1]; ++o)
            slot_pe[size_t(tile_sbeg[ti]) + owned_slot[o]] |= int(0x80000000u);
    // node graph in-edges (for the warm-start network's backward message passing)
    std::vector<int> in_beg(nn + 1, 0), in_src, out_cnt(nn, 0);
    {
        std::vector<std::vector<int>> ins(nn);
        for (int k = 0; k < nn; ++k)
            for (int e = 0; e < 8; ++e) {
                int l = edst[size_t(e) * nn + k];
                if (l >= 0) { ins[l].push_back(k); out_cnt[k]++; }
            }
        for (int l = 0; l < nn; ++l) {
            std::sort(ins[l].begin(), ins[l].end());
            in_src.insert(in_src.end(), ins[l].begin(), ins[l].end());
            in_beg[l + 1] = int(in_src.size());
        }
    }
    std::vector<float> plan_w(size_t(4) * nv);
    for (int p = 0; p < nv; ++p)
        for (int j = 0; j < 4; ++j) plan_w[size_t(j) * nv + p] = bw[size_t(j) * nv + plan_vid[p]];

    Blob blob;
    size_t o_tri = blob.add(tri), o_nvtx = blob.add(nvtx), o_bidx = blob.add(bidx), o_bw = blob.add(bw),
           o_edst = blob.add(edst), o_pvid = blob.add(plan_vid), o_ppos = blob.add(plan_pos),
           o_pw = blob.add(plan_w), o_pslot = blob.add(plan_slot), o_tvb = blob.add(tile_vbeg),
           o_tsb = blob.add(tile_sbeg), o_snode = blob.add(slot_node), o_tob = blob.add(tile_obeg),
           o_onode = blob.add(owned_node), o_oslot = blob.add(owned_slot), o_oes = blob.add(owned_eslot),
           o_lb = blob.add(list_beg), o_li = blob.add(list_idx), o_npb = blob.add(node_pbeg),
           o_npi = blob.add(node_pidx), o_vfb = blob.add(vf_beg), o_vff = blob.add(vf_face),
           o_me = blob.add(medge), o_ib = blob.add(in_beg), o_is = blob.add(in_src), o_oc = blob.add(out_cnt),
           o_sd = blob.add(slot_dest), o_pcp = blob.add(plan_cpos), o_ocp = blob.add(owned_cpos),
           o_spb = blob.add(slot_pb), o_spe = blob.add(slot_pe);
    void *mem = nullptr;
    hipError_t e = hipMalloc(&mem, blob.bytes.size());
    if (e != hipSuccess) return fail(CAPTURE_ENOMEM, "template: device allocation failed");
    e = hipMemcpy(mem, blob.bytes.data(), blob.bytes.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) { (void)hipFree(mem); return fail(CAPTURE_EHIP, "template: upload failed"); }
    auto at = [&](size_t off) { return static_cast<uint8_t *>(mem) + off; };
    capture_template *t = new capture_template;
    TemplateDev &D = t->dev;
    D.nv = nv; D.nf = nf; D.nn = nn; D.ntiles = nt; D.nslots = int(slot_node.size()); D.nmedges = nme;
    D.max_slots = max_slots; D.max_contrib = max_contrib;
    D.tri = (const int *)at(o_tri); D.node_vertex = (const int *)at(o_nvtx);
    D.bind_idx = (const int *)at(o_bidx); D.bind_w = (const float *)at(o_bw);
    D.edge_dst = (const int *)at(o_edst); D.plan_vid = (const int *)at(o_pvid);
    D.plan_pos = (const int *)at(o_ppos); D.plan_w = (const float *)at(o_pw);
    D.plan_slot = (const uint32_t *)at(o_pslot); D.tile_vbeg = (const int *)at(o_tvb);
    D.tile_sbeg = (const int *)at(o_tsb); D.slot_node = (const int *)at(o_snode);
    D.tile_obeg = (const int *)at(o_tob); D.owned_node = (const int *)at(o_onode);
    D.owned_slot = (const uint8_t *)at(o_oslot); D.owned_eslot = (const uint8_t *)at(o_oes);
    D.list_beg = (const int *)at(o_lb); D.list_idx = (const uint16_t *)at(o_li);
    D.node_pbeg = (const int *)at(o_npb); D.node_pidx = (const int *)at(o_npi);
    D.vf_beg = (const int *)at(o_vfb); D.vf_face = (const int *)at(o_vff); D.medge = (const int *)at(o_me);
    D.slot_dest = (const int *)at(o_sd);
    D.slot_pb = (const int *)at(o_spb); D.slot_pe = (const int *)at(o_spe);
    D.plan_cpos = (const uint16_t *)at(o_pcp);
    D.owned_cpos = (const uint32_t *)at(o_ocp);
    D.in_beg = (const int *)at(o_ib); D.in_src = (const int *)at(o_is); D.out_cnt = (const int *)at(o_oc);
    t->vertices_per_tile = vcap;
    t->tile_ranges.resize(size_t(6) * nt);
    for (int i = 0; i < nt; ++i) {
        int *r = t->tile_ranges.data() + size_t(6) * i;
        r[0] = tile_vbeg[i]; r[1] = tile_vbeg[i + 1] - tile_vbeg[i];
        r[2] = tile_sbeg[i]; r[3] = tile_sbeg[i + 1] - tile_sbeg[i];
        r[4] = tile_obeg[i]; r[5] = tile_obeg[i + 1] - tile_obeg[i];
    }
    t->mem = mem;
    t->bytes = blob.bytes.size();
    t->device = device;
    *out = t;
    return CAPTURE_OK;
}

// Topology-only template (no deformation graph): the mesh tables that the
// per-frame raster and decision kernels read, with the identity vertex order.
int build_topology_template(const int *tri_dev, int nv, int nf, capture_template **out, int device) {
    if (nv < 1 || nf < 1) return fail(CAPTURE_EINVAL, "mesh: need n_vertices >= 1 and n_triangles >= 1");
    if (!tri_dev) return fail(CAPTURE_EINVAL, "mesh: null triangle array");
    std::vector<int> tri;
    int rc;
    if ((rc = copy_down(tri, tri_dev, size_t(3) * nf))) return rc;
    for (int v : tri) if (v < 0 || v >= nv) return fail(CAPTURE_EINVAL, "mesh: triangle index out of range");
    std::vector<int> medge, vf_beg, vf_face, ident(nv);
    int nme = 0;
    if ((rc = topology(tri, nv, nf, medge, nme, vf_beg, vf_face))) return rc;
    for (int v = 0; v < nv; ++v) ident[v] = v;
    Blob blob;
    size_t o_tri = blob.add(tri), o_id = blob.add(ident), o_vfb = blob.add(vf_beg), o_vff = blob.add(vf_face),
           o_me = blob.add(medge);
    void *mem = nullptr;
    if (hipMalloc(&mem, blob.bytes.size()) != hipSuccess) return fail(CAPTURE_ENOMEM, "mesh: device allocation failed");
    if (hipMemcpy(mem, blob.bytes.data(), blob.bytes.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(mem);
        return fail(CAPTURE_EHIP, "mesh: upload failed");
    }
    auto at = [&](size_t off) { return static_cast<uint8_t *>(mem) + off; };
    capture_template *t = new capture_template{};
    TemplateDev &D = t->dev;
    D.nv = nv; D.nf = nf; D.nn = 0; D.nmedges = nme;
    D.tri = (const int *)at(o_tri);
    D.plan_vid = (const int *)at(o_id); D.plan_pos = (const int *)at(o_id);
    D.vf_beg = (const int *)at(o_vfb); D.vf_face = (const int *)at(o_vff); D.medge = (const int *)at(o_me);
    t->mem = mem;
    t->bytes = blob.bytes.size();
    t->device = device;
    *out = t;
    return CAPTURE_OK;
}

}  // namespace cap
