// Gauss-Newton / PCG kernels of the non-rigid stage (Sec. 3.4 energy, Sec. 4
// solver).  Tile kernels (one block per tile of every problem, from a
// host-built list of tile descriptors) stream the
// plan-ordered vertices once and accumulate per-node 6-vectors in LDS; node
// kernels (one workgroup per problem) finish the per-node sums in a fixed
// order and run the PCG vector updates with float64 dot products.
#include "device.hpp"

namespace cap {

// Work item of a block when consecutive blocks go to the accelerator dies
// (XCDs) in turn: block b runs on die b % 8, so die x is given the x-th
// contiguous eighth of the items and neighbouring tiles (which share slot
// nodes) meet in the same L2.  The grid is a multiple of 8.
__device__ inline int xcd_item(int b, int grid) { return (b & 7) * (grid >> 3) + (b >> 3); }

// The tile's contributions are stored component-major, C[comp][position],
// where each vertex binding and regulariser edge end has a fixed position
// (plan_cpos, owned_cpos) inside its slot's contiguous range, in ascending
// contribution order; every slot sum therefore reads one contiguous run
// [lbeg[s], lbeg[s + 1]), in a fixed order.
__device__ inline float run_sum(const float *__restrict__ c, int b, int e) {
    float acc = 0.0f;
    int q = b;
    for (; q + 8 <= e; q += 8) {       // eight LDS reads in flight, then the adds in order
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = c[q + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; q < e; ++q) acc += c[q];
    return acc;
}

// A slot's node in the product kernel's LDS: five float4 (R row-major, the
// node position, p; two floats of padding), read with 16-byte loads.
constexpr int kSlotRec = 20;

__device__ inline void slot_rec(const float4 *S, int sl, float R[9], float g[3], float p[6]) {
    const float4 a = S[5 * sl], b = S[5 * sl + 1], c = S[5 * sl + 2], d = S[5 * sl + 3], e = S[5 * sl + 4];
    R[0] = a.x; R[1] = a.y; R[2] = a.z; R[3] = a.w; R[4] = b.x; R[5] = b.y; R[6] = b.z; R[7] = b.w; R[8] = c.x;
    g[0] = c.y; g[1] = c.z; g[2] = c.w;
    p[0] = d.x; p[1] = d.y; p[2] = d.z; p[3] = d.w; p[4] = e.x; p[5] = e.y;
}

// A slot's node in the linearisation's LDS: four float4 (R row-major, t, the
// node position; one float of padding).
constexpr int kSlotRecLin = 16;

__device__ inline void slot_rec_lin(const float4 *S, int sl, float R[9], float t[3], float g[3]) {
    const float4 a = S[4 * sl], b = S[4 * sl + 1], c = S[4 * sl + 2], d = S[4 * sl + 3];
    R[0] = a.x; R[1] = a.y; R[2] = a.z; R[3] = a.w; R[4] = b.x; R[5] = b.y; R[6] = b.z; R[7] = b.w; R[8] = c.x;
    t[0] = c.y; t[1] = c.z; t[2] = c.w;
    g[0] = d.x; g[1] = d.y; g[2] = d.z;
}

__device__ inline void rot_apply(const float *R, const float d[3], float q[3]) {
    q[0] = (R[0] * d[0] + R[1] * d[1]) + R[2] * d[2];
    q[1] = (R[3] * d[0] + R[4] * d[1]) + R[5] * d[2];
    q[2] = (R[6] * d[0] + R[7] * d[1]) + R[8] * d[2];
}

// ----------------------------------------------------------------------------
// Linearisation: residuals, per-vertex condensed normal-equation blocks
// H_i = sum |b| G^T G (3x3) and g_i = sum b G^T r, the energy, and per-slot
// partial sums of the right-hand side -J^T B F and of diag(J^T |B| J).
// mode bit 0: energy only; bit 1: run only if the warm start rejected its
// prediction (scal[5] set), i.e. relinearise at the restored start.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(kTileThreads) void k_linearize(const ProbDev *__restrict__ P,
                                                            const TileDesc *__restrict__ D, int mode) {
    extern __shared__ float lds[];
    __shared__ double red[kTileThreads / 64][kTerms];
    __shared__ int lbeg[kMaxTileSlots + 1];
    __shared__ int ldest[kMaxTileSlots];
    const TileDesc d = D[xcd_item(blockIdx.x, gridDim.x)];
    if (d.prob < 0) return;
    const ProbDev &pr = P[d.prob];
    const TemplateDev &T = pr.T;
    const int tile = d.tile;
    const bool full = (mode & 1) == 0;
    const int nv = T.nv, nn = T.nn;
    const int vb = d.vb, nvt = d.nvt, sb = d.sb, ns = d.ns, ob = d.ob, nown = d.nown;
    // Every global read that needs no other global value first (the vertex's
    // own data, slot nodes, run offsets, destinations, owned edges), then the
    // slot nodes' state; the stop tests sit between the two rounds.  The
    // first round is branch-free: every thread loads at clamped (in-bounds)
    // positions and replaces what lies outside its ranges afterwards, so all
    // of its loads are in flight together.
    static_assert(kMaxTileSlots < kTileThreads, "one thread per slot and run offset");
    const int lv = threadIdx.x, p = vb + lv;
    const bool has_v = lv < nvt, has_s = lv < ns, has_e = lv < nown * 8;
    const int pv = min(p, nv - 1), ps = min(sb + lv, T.nslots - 1), pl = min(sb + lv, T.nslots);
    const int po = min(ob + (lv >> 3), nn - 1), pe8 = (lv & 7) * nn + po;
    uint8_t code = pr.vcode[pv];
    uint32_t packed = T.plan_slot[pv];
    float v[3], w[4], pcol[3], pva[3];
    int cp[4];
    v[0] = pr.px[pv]; v[1] = pr.px[nv + pv]; v[2] = pr.px[2 * nv + pv];
#pragma unroll
    for (int j = 0; j < 4; ++j) w[j] = T.plan_w[size_t(j) * nv + pv];
#pragma unroll
    for (int c = 0; c < 3; ++c) pcol[c] = pr.pc[size_t(c) * nv + pv];
#pragma unroll
    for (int a = 0; a < 3; ++a) pva[a] = pr.pva[size_t(a) * nv + pv];
#pragma unroll
    for (int j = 0; j < 4; ++j) cp[j] = T.plan_cpos[size_t(j) * nv + pv];
    int snode = T.slot_node[ps];
    const int sdest = T.slot_dest[ps];
    const int lb = T.list_beg[pl];
    int e_so = T.owned_slot[po], e_se = T.owned_eslot[pe8];
    uint32_t e_cp = T.owned_cpos[pe8];
    const int l0 = T.list_beg[sb];
    const double stopped = pr.scal[2], rejected = pr.scal[5];     // read here, tested below
    // the destinations and run offsets are consumed here, unconditionally, so
    // that their loads are not moved into the branches below (behind the rest)
    __asm__ volatile("" ::"v"(sdest), "v"(lb));
    if (!has_v) {
        code = 0;
        packed = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) v[a] = pcol[a] = pva[a] = 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            w[j] = 0.0f;
            cp[j] = 0;
        }
    }
    if (!full)
#pragma unroll
        for (int j = 0; j < 4; ++j) cp[j] = 0;
    if (!has_s) snode = 0;
    if (!has_e) {
        e_so = 0;
        e_se = 255;
        e_cp = 0;
    }
    if (full && has_s) ldest[lv] = sdest;
    if (full && lv <= ns) lbeg[lv] = lb - l0;
    if (stopped != 0.0) return;
    if ((mode & 2) && rejected == 0.0) return;      // conditional pass: only after a rejected prediction
    // LDS: one 64-byte record per slot (R, t, node position: four float4),
    // then contributions [12][NC]
    float4 *S = reinterpret_cast<float4 *>(lds);
    float *Cl = lds + kSlotRecLin * ns;
    if (has_s) {      // R, t and position of the slot's node
        float sv[16];
#pragma unroll
        for (int q = 0; q < 12; ++q) sv[q] = pr.state[size_t(q) * nn + snode];
#pragma unroll
        for (int q = 0; q < 3; ++q) sv[12 + q] = pr.gpos[size_t(q) * nn + snode];
        sv[15] = 0.0f;
#pragma unroll
        for (int q = 0; q < 4; ++q) S[4 * lv + q] = make_float4(sv[4 * q], sv[4 * q + 1], sv[4 * q + 2], sv[4 * q + 3]);
    }
    __syncthreads();
    // component stride of the contribution buffer: odd, so that the twelve
    // components of one position sit in different LDS banks
    const int NC = full ? (lbeg[ns] | 1) : 0;

    double e_ph = 0.0, e_s = 0.0, e_sa = 0.0, e_a = 0.0, e_v = 0.0;
    if (has_v) {
        float Hm[6] = {0, 0, 0, 0, 0, 0}, gi[3] = {0, 0, 0};
        float q[4][3];
        int sl[4];
        // the deformed position and its projection in float64: an image
        // coordinate of ~1e3 px in float32 is only good to ~1e-4 px, which the
        // photometric and silhouette residuals would feel
        double V[3] = {0, 0, 0};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            sl[j] = (packed >> (8 * j)) & 0xff;
            float Rm[9], tt[3], g[3];
            slot_rec_lin(S, sl[j], Rm, tt, g);
            const double dd[3] = {double(v[0]) - g[0], double(v[1]) - g[1], double(v[2]) - g[2]};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double qa = (double(Rm[3 * a]) * dd[0] + double(Rm[3 * a + 1]) * dd[1]) + double(Rm[3 * a + 2]) * dd[2];
                q[j][a] = float(qa);
                V[a] += double(w[j]) * ((qa + g[a]) + tt[a]);
            }
        }
        if ((code & 3) && V[2] > 0.0) {
            const double izd = 1.0 / V[2];
            const double ud = double(pr.fx) * V[0] * izd + pr.cx, vd = double(pr.fy) * V[1] * izd + pr.cy;
            int cu, cv;
            float fu, fv;
            cell_of(ud, cu, fu);
            cell_of(vd, cv, fv);
            const float iz = float(izd), X = float(V[0]), Y = float(V[1]);
            // d(u, v)/dV
            const float P0[3] = {pr.fx * iz, 0.0f, -pr.fx * X * iz * iz};
            const float P1[3] = {0.0f, pr.fy * iz, -pr.fy * Y * iz * iz};
            if (code & 1) {
                float val[3], gu[3], gv[3];
                sample_cubic3_cell(pr.blurred.g(), pr.W, pr.H, cu, fu, cv, fv, val, gu, gv);
                float res[3], n2 = 0.0f;
                for (int c = 0; c < 3; ++c) {
                    res[c] = val[c] - pcol[c];
                    n2 += res[c] * res[c];
                }
                if (!(sqrtf(n2) > pr.tau)) {
                    for (int c = 0; c < 3; ++c) {
                        const float r = pr.sw_photo * res[c];
                        float G[3];
                        for (int a = 0; a < 3; ++a) G[a] = pr.sw_photo * (gu[c] * P0[a] + gv[c] * P1[a]);
                        Hm[0] += G[0] * G[0]; Hm[1] += G[0] * G[1]; Hm[2] += G[0] * G[2];
                        Hm[3] += G[1] * G[1]; Hm[4] += G[1] * G[2]; Hm[5] += G[2] * G[2];
                        for (int a = 0; a < 3; ++a) gi[a] += G[a] * r;
                        e_ph += double(r) * double(r);
                    }
                }
            }
            if (code & 2) {
                float gu, gv;
                const float dval = sample_cubic_cell(pr.dt.g(), pr.W, pr.H, cu, fu, cv, fv, gu, gv);
                const float r = pr.sw_sil * dval;
                const float b = (code & 4) ? -1.0f : 1.0f;
                float G[3];
                for (int a = 0; a < 3; ++a) G[a] = pr.sw_sil * (gu * P0[a] + gv * P1[a]);
                Hm[0] += G[0] * G[0]; Hm[1] += G[0] * G[1]; Hm[2] += G[0] * G[2];
                Hm[3] += G[1] * G[1]; Hm[4] += G[1] * G[2]; Hm[5] += G[2] * G[2];
                for (int a = 0; a < 3; ++a) gi[a] += b * G[a] * r;
                e_s += double(b) * double(r) * double(r);
                e_sa += double(r) * double(r);
            }
        }
        if (code & 8) {   // velocity prior: r = sqrt(w_vel) (V - V_anchor), dr/dV = sqrt(w_vel) I
            for (int a = 0; a < 3; ++a) {
                const double dv = V[a] - double(pva[a]);
                gi[a] += float(double(pr.w_vel) * dv);
                e_v += double(pr.w_vel) * dv * dv;
            }
            Hm[0] += pr.w_vel; Hm[3] += pr.w_vel; Hm[5] += pr.w_vel;
        }
        if (full) {
            if (code & 11)
                for (int q6 = 0; q6 < 6; ++q6) pr.Hm[size_t(q6) * nv + p] = Hm[q6];
            // contributions to the 4 bound nodes: rhs -w[q x g; g], diag w^2[diag(Q^T H Q); diag(H)]
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float *c = Cl + cp[j];
                const float *qq = q[j];
                const float ww = w[j], w2 = w[j] * w[j];
                float qxg[3];
                cross3(qq, gi, qxg);
                c[0] = -ww * qxg[0]; c[NC] = -ww * qxg[1]; c[2 * NC] = -ww * qxg[2];
                c[3 * NC] = -ww * gi[0]; c[4 * NC] = -ww * gi[1]; c[5 * NC] = -ww * gi[2];
                const float xx = Hm[0], xy = Hm[1], xz = Hm[2], yy = Hm[3], yz = Hm[4], zz = Hm[5];
                c[6 * NC] = w2 * ((qq[2] * qq[2] * yy - 2.0f * qq[2] * qq[1] * yz) + qq[1] * qq[1] * zz);
                c[7 * NC] = w2 * ((qq[2] * qq[2] * xx - 2.0f * qq[2] * qq[0] * xz) + qq[0] * qq[0] * zz);
                c[8 * NC] = w2 * ((qq[1] * qq[1] * xx - 2.0f * qq[1] * qq[0] * xy) + qq[0] * qq[0] * yy);
                c[9 * NC] = w2 * xx; c[10 * NC] = w2 * yy; c[11 * NC] = w2 * zz;
            }
        }
    }
    // regulariser edges owned by this tile: r = sqrt(w)(R_k(g_l - g_k) + g_k + t_k - g_l - t_l)
    for (int idx = lv; idx < nown * 8; idx += kTileThreads) {
        const int o = idx >> 3, e = idx & 7;
        const int so = idx == lv ? e_so : T.owned_slot[ob + o];
        const int se = idx == lv ? e_se : T.owned_eslot[size_t(e) * nn + ob + o];
        if (se == 255) continue;
        const uint32_t cpe = idx == lv ? e_cp : T.owned_cpos[size_t(e) * nn + ob + o];
        float *c0 = Cl + (cpe & 0xffffu), *c1 = Cl + (cpe >> 16);
        float Rk[9], tk[3], gk[3], Rl[9], tl[3], gl[3];
        slot_rec_lin(S, so, Rk, tk, gk);
        slot_rec_lin(S, se, Rl, tl, gl);
        float d[3] = {gl[0] - gk[0], gl[1] - gk[1], gl[2] - gk[2]};
        float ekl[3];
        rot_apply(Rk, d, ekl);
        float r[3];
        {
            const double dd[3] = {double(gl[0]) - gk[0], double(gl[1]) - gk[1], double(gl[2]) - gk[2]};
            for (int a = 0; a < 3; ++a) {
                const double ed = (double(Rk[3 * a]) * dd[0] + double(Rk[3 * a + 1]) * dd[1]) + double(Rk[3 * a + 2]) * dd[2];
                r[a] = float(double(pr.sw_arap) * ((ed - dd[a]) + (double(tk[a]) - tl[a])));
            }
        }
        e_a += double(r[0]) * r[0] + double(r[1]) * r[1] + double(r[2]) * r[2];
        if (full) {
            float exr[3];
            cross3(ekl, r, exr);
            const float s = pr.sw_arap, wa = pr.w_arap;
            c0[0] = -s * exr[0]; c0[NC] = -s * exr[1]; c0[2 * NC] = -s * exr[2];
            c0[3 * NC] = -s * r[0]; c0[4 * NC] = -s * r[1]; c0[5 * NC] = -s * r[2];
            c0[6 * NC] = wa * (ekl[1] * ekl[1] + ekl[2] * ekl[2]);
            c0[7 * NC] = wa * (ekl[0] * ekl[0] + ekl[2] * ekl[2]);
            c0[8 * NC] = wa * (ekl[0] * ekl[0] + ekl[1] * ekl[1]);
            c0[9 * NC] = wa; c0[10 * NC] = wa; c0[11 * NC] = wa;
            c1[0] = 0.0f; c1[NC] = 0.0f; c1[2 * NC] = 0.0f;
            c1[3 * NC] = s * r[0]; c1[4 * NC] = s * r[1]; c1[5 * NC] = s * r[2];
            c1[6 * NC] = 0.0f; c1[7 * NC] = 0.0f; c1[8 * NC] = 0.0f;
            c1[9 * NC] = wa; c1[10 * NC] = wa; c1[11 * NC] = wa;
        }
    }
    __syncthreads();
    if (full) {
        for (int pair = threadIdx.x; pair < ns * 12; pair += blockDim.x) {
            const int s = pair / 12, comp = pair - s * 12;
            pr.partial[size_t(comp) * T.nslots + ldest[s]] = run_sum(Cl + comp * NC, lbeg[s], lbeg[s + 1]);
        }
    }
    double es[kTerms] = {e_ph, e_s, e_sa, e_a, e_v};
    block_sum_n<kTileThreads, kTerms>(es, red);
    if (threadIdx.x == 0) {
        CAP_GLOBAL double *te = pr.tile_e.g() + size_t(tile) * kTerms;
        for (int q = 0; q < kTerms; ++q) te[q] = es[q];
    }
}

// ----------------------------------------------------------------------------
// Matrix-free J^T |B| J v per tile: dV_i = sum_j w_j (w_k x q_j + tau_k),
// f_i = H_i dV_i, node contributions w_j [q_j x f_i; f_i]; regulariser edges
// u = w_k x e_kl + tau_k - tau_l add w_a [e x u; u] to k and w_a [0; -u] to l.
// Per-tile partial sums, one per (tile, slot node); the nodes add their
// partials in tile order.  The PCG vectors are float64, the product float32.
//
// The launch also holds the vector step of Jacobi-preconditioned CG
// (M = diag(A)^-1) that precedes the product, for the nodes of the tile's
// slots: the tile that owns a node stores its new vectors, the others compute
// the same values for their own use.  Two arrangements of the iteration:
//
// kCgFused (Chronopoulos-Gear; one launch per iteration).  The two inner
// products of an iteration, r.u and u.Au, are both known before the next
// vector step: each tile sums its share (r.u over the nodes it owns, u.Au
// over its slot partials), and every workgroup of the next launch adds the
// tile sums in the same fixed order, so all of them form the same scalars.
// With u_0 = M r_0 and p_{-1} = s_{-1} = 0, launch j >= 1 forms
//   gamma = r_{j-1}.u_{j-1},  delta = u_{j-1}.A u_{j-1},
//   beta = gamma / gamma_{j-2} (0 for j = 1),  den = delta - beta gamma / alpha_{j-2} (= p.Ap),
//   alpha = gamma / den, and stops (x stays x_{j-1}) if den <= 0 or gamma == 0;
//   p_{j-1} = u_{j-1} + beta p_{j-2},  s_{j-1} = A u_{j-1} + beta s_{j-2} (= A p_{j-1}),
//   x_j = x_{j-1} + alpha p_{j-1},  r_j = r_{j-1} - alpha s_{j-1},  u_j = M r_j,
// then multiplies u_j; launch 0 only multiplies u_0.  In exact arithmetic
// these are the iterates of the standard recurrence; in floating point the
// recurrence for s = A p lets rounding accumulate, so this arrangement serves
// short schedules (k_cg_finish completes the last iteration).
//
// kCgStandard (two launches per iteration, with k_pcg_node).  Launch j forms
// p_j = u_j + beta_{j-1} p_{j-1} (beta from the r.u sums of k_pcg_node's
// blocks; p_0 = u_0) and multiplies it, summing p_j.Ap_j per tile; k_pcg_node
// then updates x, r and u from the complete A p_j.  Used for large grids
// (fewer registers, no per-tile redundancy beyond p) and long schedules.
//
// j < 0 (either mode): multiply the vector p of capture_linearize.
// Vectors of generation m live in buffer m & 1 (fused: x, r, u of launch j in
// j & 1, its p and s in (j - 1) & 1; standard: p_j in j & 1), and the partials
// of fused launch j in components 6 (j & 1) .. 6 (j & 1) + 5 of `partial`, so
// no launch writes what another workgroup of the same launch reads.
// ----------------------------------------------------------------------------
// Partials of a node read together (a node is touched by a handful of tiles;
// further ones, if any, one after another).
constexpr int kParts = 8;
constexpr int kCgFused = 0, kCgStandard = 1;

// (component, slot) items per thread whose loads are in flight together: two
// for grids the chip holds at once, one (fewer registers, more workgroups
// per CU) for larger grids
template <int kSplit>
constexpr int cg_group() { return kSplit ? 1 : 2; }

template <int kSplit, int kMode>
__global__ __launch_bounds__(kTileThreads) void k_cg(const ProbDev *__restrict__ P, const TileDesc *__restrict__ D, int j) {
    extern __shared__ float lds[];
    __shared__ int lbeg[kMaxTileSlots + 1];
    __shared__ int ldest[kMaxTileSlots];
    constexpr int kCgGroup = cg_group<kSplit>();
    constexpr bool kFused = kMode == kCgFused;
    __shared__ double red[kTileThreads / 64][3];
    __shared__ float psum[6][kMaxTileSlots];      // the slot sums (for u.Au / p.Ap in one fixed order)
    const TileDesc d = D[xcd_item(blockIdx.x, gridDim.x)];
    if (d.prob < 0) return;
    const ProbDev &pr = P[d.prob];
    const TemplateDev &T = pr.T;
    const int nv = T.nv, nn = T.nn, ns = d.ns, nown = d.nown, nt = T.ntiles;
    // Global reads come in two dependent rounds: indices (vertex codes and
    // contribution positions, slot nodes, run offsets, destinations, owned
    // edges, the vector items' nodes and partial ranges, the previous
    // launches' sums) and then the data they select; the stop flag is tested
    // between.  The first round is branch-free: every thread loads at clamped
    // (in-bounds) positions and replaces what lies outside its ranges
    // afterwards, so all of its loads are in flight together.
    static_assert(kMaxTileSlots < kTileThreads, "one thread per slot and run offset");
    const int lv = threadIdx.x, p = d.vb + lv;
    const bool has_v = lv < d.nvt, has_s = lv < ns, has_e = lv < nown * 8;
    const int pv = min(p, nv - 1), ps = min(d.sb + lv, T.nslots - 1), pl = min(d.sb + lv, T.nslots);
    const int po = min(d.ob + (lv >> 3), nn - 1), pe8 = (lv & 7) * nn + po;
    uint8_t code = pr.vcode[pv];
    int cp[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) cp[q] = T.plan_cpos[size_t(q) * nv + pv];
    int snode = T.slot_node[ps];
    const int sdest = T.slot_dest[ps];
    const int lb = T.list_beg[pl];
    int e_so = T.owned_slot[po], e_se = T.owned_eslot[pe8];
    uint32_t e_cp = T.owned_cpos[pe8];
    const int l0 = T.list_beg[d.sb];
    // vector items: item i = c * ns + s (component c of slot s's node)
    const int nsv = max(ns, 1), nitems = 6 * ns;
    int in_node[kCgGroup], in_pb[kCgGroup], in_pe[kCgGroup];
    auto item_index = [&](int g0) {
#pragma unroll
        for (int m = 0; m < kCgGroup; ++m) {
            const int i = min(g0 + lv + m * kTileThreads, max(nitems - 1, 0));
            const int c = i / nsv, gs = min(d.sb + (i - c * nsv), T.nslots - 1);
            in_node[m] = T.slot_node[gs];
            in_pe[m] = T.slot_pe[gs];
            if (kFused) in_pb[m] = T.slot_pb[gs];
        }
    };
    item_index(0);
    // the previous launches' sums, formed identically by every wave: fused,
    // the tiles' r.u, u.Au and r.r of launch j - 1; standard, the node
    // blocks' r.u and r.r of k_pcg_node j - 1
    double tsum[3] = {0.0, 0.0, 0.0};
    if (j >= 1) {
        if (kFused) {
            wave_sum_n<3>(pr.dots.g() + size_t((j - 1) & 1) * 3 * nt, nt, nt, tsum);
        } else {
            const int nb = (nn + 255) / 256;
            double ns2[2];
            wave_sum_n<2>(pr.nsum.g() + size_t((j - 1) & 1) * 2 * nb, nb, nb, ns2);
            tsum[0] = ns2[0];
            tsum[2] = ns2[1];
        }
    }
    const double pcg_stopped = pr.scal[1];     // read here, tested below
    // the destinations and run offsets are consumed here, unconditionally, so
    // that their loads are not moved into the branches below (behind the rest)
    __asm__ volatile("" ::"v"(sdest), "v"(lb));
    if (!has_v) {
        code = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) cp[q] = 0;
    }
    if (!has_s) snode = 0;
    if (!has_e) {
        e_so = 0;
        e_se = 255;
        e_cp = 0;
    }
    if (has_s) ldest[lv] = sdest;
    if (lv <= ns) lbeg[lv] = lb - l0;
    if (pcg_stopped != 0.0) return;    // this problem's PCG has stopped
    const bool act = (code & 11) != 0;
    uint32_t packed = 0;
    float v[3] = {0, 0, 0}, w[4] = {0, 0, 0, 0}, Hm[6] = {0, 0, 0, 0, 0, 0};
    if (act) {
        packed = T.plan_slot[p];
        v[0] = pr.px[p]; v[1] = pr.px[nv + p]; v[2] = pr.px[2 * nv + p];
#pragma unroll
        for (int q = 0; q < 4; ++q) w[q] = T.plan_w[size_t(q) * nv + p];
#pragma unroll
        for (int q6 = 0; q6 < 6; ++q6) Hm[q6] = pr.Hm[size_t(q6) * nv + p];
    }
    // LDS: one 80-byte record per slot (R, node position, the vector
    // multiplied: five float4), then contributions [3][NC] (kSplit) or [6][NC]
    float4 *S = reinterpret_cast<float4 *>(lds);
    float *Sf = lds;
    float *C = lds + kSlotRec * ns;
    if (has_s) {      // R and position of the slot's node
        float sv[12];
#pragma unroll
        for (int q = 0; q < 9; ++q) sv[q] = pr.state[size_t(q) * nn + snode];
#pragma unroll
        for (int q = 0; q < 3; ++q) sv[9 + q] = pr.gpos[size_t(q) * nn + snode];
#pragma unroll
        for (int q = 0; q < 3; ++q) S[5 * lv + q] = make_float4(sv[4 * q], sv[4 * q + 1], sv[4 * q + 2], sv[4 * q + 3]);
        Sf[kSlotRec * lv + 18] = 0.0f;
        Sf[kSlotRec * lv + 19] = 0.0f;
    }
    // the vector step, one group of items at a time (one group unless the
    // tile has more than kCgGroup * kTileThreads / 6 slots)
    const int gp = (j - 1) & 1;                      // generation j - 1
    double gam = 0.0, rr = 0.0;                      // fused: owned r_j . u_j and r_j . r_j
    double alpha = 0.0, beta = 0.0;
    for (int g0 = 0; g0 < nitems; g0 += kCgGroup * kTileThreads) {
        if (g0 > 0) item_index(g0);
        float iv[kCgGroup];                          // j < 0: the vector to multiply
        double iu[kCgGroup], ir[kCgGroup], ix[kCgGroup], ipo[kCgGroup], iso[kCgGroup];
        float idi[kCgGroup];
        float ipart[kCgGroup][kParts];
#pragma unroll
        for (int m = 0; m < kCgGroup; ++m) {
            const int i = min(g0 + lv + m * kTileThreads, max(nitems - 1, 0));
            const int c = i / nsv;
            const size_t o = size_t(c) * nn + in_node[m];
            if (j < 0) {
                iv[m] = pr.p[o];
            } else if (!kFused) {                    // u_j and p_{j-1}
                iu[m] = pr.vu[j & 1][o];
                if (j >= 1) ipo[m] = pr.vp[gp][o];
            } else if (j == 0) {
                iu[m] = pr.vu[0][o];
            } else {
                iu[m] = pr.vu[gp][o]; ir[m] = pr.vr[gp][o]; ix[m] = pr.vx[gp][o]; idi[m] = pr.dinv[o];
                if (j >= 2) { ipo[m] = pr.vp[j & 1][o]; iso[m] = pr.vs[j & 1][o]; }
                const int pe = in_pe[m] & 0x7fffffff, qmax = max(pe - 1, 0);
                const CAP_GLOBAL float *pp = pr.partial.g() + size_t(6 * gp + c) * T.nslots;
#pragma unroll
                for (int q = 0; q < kParts; ++q) ipart[m][q] = pp[min(in_pb[m] + q, qmax)];
            }
        }
        if (j >= 1 && g0 == 0) {
            // the scalars (the same in every workgroup)
            const double bb = pr.cg[5];
            if (kFused) {       // iteration j - 1
                const double gamma = j == 1 ? pr.scal[0] : tsum[0], delta = tsum[1];
                const double rho = j == 1 ? bb : tsum[2];
                double den = delta;
                if (j >= 2) {
                    const CAP_GLOBAL double *cg = pr.cg.g() + 2 * gp;
                    beta = gamma / cg[0];
                    den = delta - beta * gamma / cg[1];
                }
                // p.Ap <= 0, r.u == 0 or ||r_{j-1}|| within the tolerance: x stays x_{j-1}
                if (den <= 0.0 || gamma == 0.0 || (pr.pcg_tol2 > 0.0 && rho <= pr.pcg_tol2 * bb)) {
                    if (d.tile == 0 && lv == 0) {
                        pr.scal[1] = 1.0;
                        pr.cg[4] = double(j - 1);
                    }
                    return;
                }
                alpha = gamma / den;
                if (d.tile == 0 && lv == 0) {
                    pr.cg[2 * (j & 1)] = gamma;
                    pr.cg[2 * (j & 1) + 1] = alpha;
                }
            } else {            // beta_{j-1} = r_j.u_j / r_{j-1}.u_{j-1}
                const double gamma = tsum[0], rho = tsum[2];
                // r.u == 0 or ||r_j|| within the tolerance: x stays x_j
                if (gamma == 0.0 || (pr.pcg_tol2 > 0.0 && rho <= pr.pcg_tol2 * bb)) {
                    if (d.tile == 0 && lv == 0) {
                        pr.scal[1] = 1.0;
                        pr.cg[4] = double(j);
                    }
                    return;
                }
                beta = gamma / pr.cg[2 * gp];
            }
        }
#pragma unroll
        for (int m = 0; m < kCgGroup; ++m) {
            const int i = g0 + lv + m * kTileThreads;
            if (i >= nitems) continue;
            const int c = i / nsv, s = i - c * nsv;
            float val;
            if (j < 0) {
                val = iv[m];
            } else if (!kFused) {
                // rounded to float32 once: the vector multiplied is the one accumulated
                const double pn = j == 0 ? iu[m] : double(float(fma(beta, ipo[m], iu[m])));
                if (in_pe[m] < 0) pr.vp[j & 1][size_t(c) * nn + in_node[m]] = pn;   // owner stores p_j
                val = float(pn);
            } else if (j == 0) {
                val = float(iu[m]);
            } else {
                const int pe = in_pe[m] & 0x7fffffff;
                float wv = 0.0f;        // A u_{j-1} of the node: its partials in order
#pragma unroll
                for (int q = 0; q < kParts; ++q)
                    if (in_pb[m] + q < pe) wv += ipart[m][q];
                for (int q = in_pb[m] + kParts; q < pe; ++q) wv += pr.partial[size_t(6 * gp + c) * T.nslots + q];
                double pn, sn;
                if (j == 1) {
                    pn = iu[m];
                    sn = double(wv);
                } else {
                    pn = fma(beta, ipo[m], iu[m]);
                    sn = fma(beta, iso[m], double(wv));
                }
                const double rn = fma(-alpha, sn, ir[m]);
                const double un = double(float(double(idi[m]) * rn));   // as multiplied
                if (in_pe[m] < 0) {        // this tile owns the node: store its vectors
                    const size_t o = size_t(c) * nn + in_node[m];
                    pr.vp[gp][o] = pn;
                    pr.vs[gp][o] = sn;
                    pr.vx[j & 1][o] = fma(alpha, pn, ix[m]);
                    pr.vr[j & 1][o] = rn;
                    pr.vu[j & 1][o] = un;
                    gam += rn * un;
                    rr += rn * rn;
                }
                val = float(un);        // the product runs in float32
            }
            Sf[kSlotRec * s + 12 + c] = val;
        }
    }
    __syncthreads();
    const int NC = lbeg[ns] | 1;     // odd component stride: components in different LDS banks
    // With kSplit the six components are reduced in two passes of three
    // (rotational, then translational) through one [3][NC] buffer, which
    // halves the LDS of a workgroup and so raises the workgroups a CU holds
    // (for grids larger than the chip); otherwise in one pass through [6][NC]
    // (shorter workgroup life, for small grids).
    float *C2 = kSplit ? C : C + 3 * NC;    // translational components
    float f[3] = {0, 0, 0};
    if (d.nvt > lv) {
        if (act) {
            float q[4][3];
            float dV[3] = {0, 0, 0};
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int sl = (packed >> (8 * b)) & 0xff;
                float R[9], g[3], pp[6];
                slot_rec(S, sl, R, g, pp);
                float dd[3] = {v[0] - g[0], v[1] - g[1], v[2] - g[2]};
                rot_apply(R, dd, q[b]);
                float oxq[3];
                cross3(pp, q[b], oxq);
#pragma unroll
                for (int a = 0; a < 3; ++a) dV[a] += w[b] * (oxq[a] + pp[3 + a]);
            }
            f[0] = (Hm[0] * dV[0] + Hm[1] * dV[1]) + Hm[2] * dV[2];
            f[1] = (Hm[1] * dV[0] + Hm[3] * dV[1]) + Hm[4] * dV[2];
            f[2] = (Hm[2] * dV[0] + Hm[4] * dV[1]) + Hm[5] * dV[2];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                float qxf[3];
                cross3(q[b], f, qxf);
                float *cj = C + cp[b];
                cj[0] = w[b] * qxf[0]; cj[NC] = w[b] * qxf[1]; cj[2 * NC] = w[b] * qxf[2];
            }
        } else {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                w[b] = 0.0f;      // zero contributions in both passes
                for (int q3 = 0; q3 < 3; ++q3) C[q3 * NC + cp[b]] = 0.0f;
            }
        }
    }
    const float wa = pr.w_arap;
    // regulariser edge k -> l: u = w_k x e_kl + tau_k - tau_l; rotational part e x u
    auto edge_u = [&](int so, int se, float ekl[3], float u[3]) {
        float Rk[9], gk[3], pk[6], Rl[9], gl[3], pl6[6];
        slot_rec(S, so, Rk, gk, pk);
        slot_rec(S, se, Rl, gl, pl6);
        float dd[3] = {gl[0] - gk[0], gl[1] - gk[1], gl[2] - gk[2]};
        rot_apply(Rk, dd, ekl);
        float oxe[3];
        cross3(pk, ekl, oxe);
        u[0] = (oxe[0] + pk[3]) - pl6[3]; u[1] = (oxe[1] + pk[4]) - pl6[4]; u[2] = (oxe[2] + pk[5]) - pl6[5];
    };
    float eu[3] = {0, 0, 0};
    for (int idx = lv; idx < nown * 8; idx += kTileThreads) {
        const int o = idx >> 3, e = idx & 7;
        const int so = idx == lv ? e_so : T.owned_slot[d.ob + o];
        const int se = idx == lv ? e_se : T.owned_eslot[size_t(e) * nn + d.ob + o];
        if (se == 255) continue;
        const uint32_t cpe = idx == lv ? e_cp : T.owned_cpos[size_t(e) * nn + d.ob + o];
        float ekl[3], u[3], exu[3];
        edge_u(so, se, ekl, u);
        cross3(ekl, u, exu);
        float *c0 = C + (cpe & 0xffffu), *c1 = C + (cpe >> 16);
        c0[0] = wa * exu[0]; c0[NC] = wa * exu[1]; c0[2 * NC] = wa * exu[2];
        c1[0] = 0.0f; c1[NC] = 0.0f; c1[2 * NC] = 0.0f;
        if (idx == lv) { eu[0] = u[0]; eu[1] = u[1]; eu[2] = u[2]; }
    }
    // partials of this launch (also kept in LDS for u.Au / p.Ap)
    const size_t pbase = size_t(j < 0 || !kFused ? 0 : 6 * (j & 1)) * T.nslots;
    if (kSplit) {
        __syncthreads();
        for (int pair = lv; pair < ns * 3; pair += kTileThreads) {
            const int s = pair / 3, comp = pair - s * 3;
            const float sum = run_sum(C + comp * NC, lbeg[s], lbeg[s + 1]);
            pr.partial[pbase + size_t(comp) * T.nslots + ldest[s]] = sum;
            psum[comp][s] = sum;
        }
        __syncthreads();
    }
    if (d.nvt > lv) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            float *cj = C2 + cp[b];
            cj[0] = w[b] * f[0]; cj[NC] = w[b] * f[1]; cj[2 * NC] = w[b] * f[2];
        }
    }
    for (int idx = lv; idx < nown * 8; idx += kTileThreads) {
        const int o = idx >> 3, e = idx & 7;
        const int se = idx == lv ? e_se : T.owned_eslot[size_t(e) * nn + d.ob + o];
        if (se == 255) continue;
        const uint32_t cpe = idx == lv ? e_cp : T.owned_cpos[size_t(e) * nn + d.ob + o];
        float u[3];
        if (idx == lv) {
            u[0] = eu[0]; u[1] = eu[1]; u[2] = eu[2];
        } else {
            float ekl[3];
            edge_u(T.owned_slot[d.ob + o], se, ekl, u);
        }
        float *c0 = C2 + (cpe & 0xffffu), *c1 = C2 + (cpe >> 16);
        c0[0] = wa * u[0]; c0[NC] = wa * u[1]; c0[2 * NC] = wa * u[2];
        c1[0] = -wa * u[0]; c1[NC] = -wa * u[1]; c1[2 * NC] = -wa * u[2];
    }
    __syncthreads();
    constexpr int kComps = kSplit ? 3 : 6;
    for (int pair = lv; pair < ns * kComps; pair += kTileThreads) {
        const int s = pair / kComps, comp = pair - s * kComps, cg = (kSplit ? 3 : 0) + comp;
        const float sum = run_sum(C + comp * NC, lbeg[s], lbeg[s + 1]);
        pr.partial[pbase + size_t(cg) * T.nslots + ldest[s]] = sum;
        psum[cg][s] = sum;
    }
    if (j >= 0) {
        // v.Av of this tile (v = u fused, p standard): each slot's six partials
        // times its node's v, in one order whichever reduction variant ran
        __syncthreads();
        if (kFused) {
            double vav = 0.0;
            if (lv < ns)
#pragma unroll
                for (int c = 0; c < 6; ++c) vav += double(Sf[kSlotRec * lv + 12 + c]) * double(psum[c][lv]);
            double ts[3] = {gam, vav, rr};
            block_sum_n<kTileThreads, 3>(ts, red);
            if (lv == 0) {
                CAP_GLOBAL double *dp = pr.dots.g() + size_t(j & 1) * 3 * nt;
                dp[d.tile] = ts[0];
                dp[nt + d.tile] = ts[1];
                dp[2 * nt + d.tile] = ts[2];
            }
        } else if (lv < 64) {      // p.Ap of the tile: the first wave adds the slots (no further barrier)
            double v = 0.0;
            for (int s = lv; s < ns; s += 64)
#pragma unroll
                for (int c = 0; c < 6; ++c) v += double(Sf[kSlotRec * s + 12 + c]) * double(psum[c][s]);
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
            if (lv == 0) pr.dots[nt + d.tile] = v;
        }
    }
}

template __global__ void k_cg<0, kCgFused>(const ProbDev *, const TileDesc *, int);
template __global__ void k_cg<0, kCgStandard>(const ProbDev *, const TileDesc *, int);
template __global__ void k_cg<1, kCgStandard>(const ProbDev *, const TileDesc *, int);

// ----------------------------------------------------------------------------
// Node kernels: one workgroup per problem.
// ----------------------------------------------------------------------------

// k_node_init: items per thread held in registers (kInitBlocks x kInitThreads
// threads: 8,192 items, 1,365 nodes); larger problems take the strided loop
constexpr int kInitItems = 2;


__device__ inline float sum_parts(gptr<const float> partial, int stride, int c, int pb, int pe) {
    float v[kParts];
#pragma unroll
    for (int u = 0; u < kParts; ++u) v[u] = pb + u < pe ? partial[size_t(c) * stride + pb + u] : 0.0f;
    float a = 0.0f;
#pragma unroll
    for (int u = 0; u < kParts; ++u)
        if (pb + u < pe) a += v[u];
    for (int q = pb + kParts; q < pe; ++q) a += partial[size_t(c) * stride + q];
    return a;
}

// The same for G items at once, without branches between the loads: every
// item's first kParts loads are issued unconditionally (positions past pe
// re-read the node's last part, part 0 for a node without parts) and in
// flight together, then the items' sums, then (rarely) their parts past
// kParts; each item's sum is formed in the same order as by sum_parts.  The
// c[] must be components (0..11).  This pays where the branchy loads
// serialise many items (k_node_init); with few parts per item the extra
// loads cost more than the waits they save (k_node_pcg).
template <int G>
__device__ inline void sum_parts_n(gptr<const float> partial, int stride, const int (&c)[G], const int (&pb)[G],
                                   const int (&pe)[G], float (&out)[G]) {
    float v[G][kParts];
#pragma unroll
    for (int h = 0; h < G; ++h) {
        const int qmax = max(pe[h] - 1, 0);
#pragma unroll
        for (int u = 0; u < kParts; ++u) v[h][u] = partial[size_t(c[h]) * stride + min(pb[h] + u, qmax)];
    }
#pragma unroll
    for (int h = 0; h < G; ++h) {
        float a = 0.0f;
#pragma unroll
        for (int u = 0; u < kParts; ++u)
            if (pb[h] + u < pe[h]) a += v[h][u];
        out[h] = a;
    }
#pragma unroll
    for (int h = 0; h < G; ++h)
        for (int q = pb[h] + kParts; q < pe[h]; ++q) out[h] += partial[size_t(c[h]) * stride + q];
}

__device__ inline float gather_node(const TemplateDev &T, gptr<const float> partial, int stride, int k,
                                    int c) {
    return sum_parts(partial, stride, c, T.node_pbeg[k], T.node_pbeg[k + 1]);
}

// After a linearisation, in two launches.  k_node_init (kInitBlocks
// workgroups per problem, blockIdx.y = problem): b, diag, Jacobi
// preconditioner and PCG start vectors (x_0 = 0, r_0 = b, u_0 = M^-1 r_0,
// generation 0) of its share of the (component, node) items, one item per
// thread, every load issued before the stop tests; its r.u and b.b sums go
// to scal[kInitPart + 2 blockIdx.x ..].  k_node_init_fin (one workgroup per
// problem) adds those sums in workgroup order and the tiles' energy sums in
// tile order, and takes the decisions: the energy of GN step `gn`, the
// scalars of the first PCG iteration and the stops.
// check_target bit 0: stop when the energy reaches the target; bit 1: the
// conditional pass (see k_linearize); bit 2: the learned start's selection
// after the linearisation at the prediction: keep the prediction only if
// its energy is below the energy in scal slot `slot_prev` (that of the
// previous frame's state), otherwise undo any stop (the schedule is again
// gn_iters steps) and restore the start state from state0; scal[4] and
// scal[6] hold the two energies, scal[5] the rejection.  With energy_only
// the first launch is left out.
__global__ __launch_bounds__(kInitThreads) void k_node_init(const ProbDev *__restrict__ P, int check_target) {
    __shared__ double red[kInitThreads / 64][2];
    const ProbDev &pr = P[blockIdx.y];
    const TemplateDev &T = pr.T;
    const int nn = T.nn, n6 = 6 * nn;
    const int gt = blockIdx.x * kInitThreads + threadIdx.x, stride = gridDim.x * kInitThreads;
    const bool regs = n6 <= kInitItems * stride;
    int pb[kInitItems], pe[kInitItems];
    if (regs) {     // unconditional loads at clamped positions, zeroed past the items
#pragma unroll
        for (int j = 0; j < kInitItems; ++j) {
            const int k = min(gt + j * stride, n6 - 1) % nn;
            pb[j] = T.node_pbeg[k]; pe[j] = T.node_pbeg[k + 1];
        }
#pragma unroll
        for (int j = 0; j < kInitItems; ++j)
            if (gt + j * stride >= n6) pb[j] = pe[j] = 0;
    }
    // stopped at the target energy (never so at the selection, which follows
    // the frame set-up's cleared flags)
    if (pr.scal[2] != 0.0 && !(check_target & 4)) return;
    if ((check_target & 2) && pr.scal[5] == 0.0) return;   // conditional pass (see k_linearize)
    double v[2] = {0.0, 0.0};      // r.u, b.b
    if (regs) {
        // items in groups of two, each group's loads (b and the diagonal,
        // kParts parts each) in flight together
        constexpr int G = 2;
        static_assert(kInitItems % G == 0, "whole groups");
#pragma unroll
        for (int g = 0; g < kInitItems; g += G) {
            if (g * stride >= n6) break;                 // (uniform) no thread has these items
            int cb[G], cd[G], gb[G], ge[G];
            float bb[G], dd[G];
#pragma unroll
            for (int h = 0; h < G; ++h) {
                cb[h] = min(gt + (g + h) * stride, n6 - 1) / nn;
                cd[h] = 6 + cb[h];
                gb[h] = pb[g + h];
                ge[h] = pe[g + h];
            }
            sum_parts_n<G>(pr.partial, T.nslots, cb, gb, ge, bb);
            sum_parts_n<G>(pr.partial, T.nslots, cd, gb, ge, dd);
#pragma unroll
            for (int h = 0; h < G; ++h) {
                const int i = gt + (g + h) * stride;
                if (i < n6) {
                    const float b = bb[h], d = dd[h];
                    const float mi = d > 0.0f ? 1.0f / d : 1.0f;
                    const double u = double(mi * b);     // float32, as multiplied
                    pr.b[i] = b; pr.diag[i] = d; pr.dinv[i] = mi;
                    pr.vx[0][i] = 0.0; pr.vr[0][i] = double(b); pr.vu[0][i] = u;
                    v[0] += double(b) * u;
                    v[1] += double(b) * double(b);
                }
            }
        }
    } else {
        for (int i = gt; i < n6; i += stride) {
            const int c = i / nn, k = i - c * nn;
            const float b = gather_node(T, pr.partial, T.nslots, k, c);
            const float d = gather_node(T, pr.partial, T.nslots, k, 6 + c);
            const float mi = d > 0.0f ? 1.0f / d : 1.0f;
            const double u = double(mi * b);     // float32, as multiplied
            pr.b[i] = b; pr.diag[i] = d; pr.dinv[i] = mi;
            pr.vx[0][i] = 0.0; pr.vr[0][i] = double(b); pr.vu[0][i] = u;
            v[0] += double(b) * u;
            v[1] += double(b) * double(b);
        }
    }
    block_sum_n<kInitThreads, 2>(v, red);
    if (threadIdx.x == 0) {
        pr.scal[kInitPart + 2 * blockIdx.x] = v[0];
        pr.scal[kInitPart + 2 * blockIdx.x + 1] = v[1];
    }
}

__global__ __launch_bounds__(kInitFinThreads) void k_node_init_fin(const ProbDev *__restrict__ P, int gn, int energy_only,
                                                                   int check_target, int slot_prev, int gn_iters,
                                                                   int nparts) {
    __shared__ double red[kInitFinThreads / 64][kTerms];
    __shared__ int reject;
    const ProbDev &pr = P[blockIdx.x];
    const TemplateDev &T = pr.T;
    double v[kTerms] = {0, 0, 0, 0, 0};   // the energy terms
    for (int t = threadIdx.x; t < T.ntiles; t += blockDim.x)
        for (int q = 0; q < kTerms; ++q) v[q] += pr.tile_e[size_t(t) * kTerms + q];
    if (pr.scal[2] != 0.0 && !(check_target & 4)) return;          // as in k_node_init
    if ((check_target & 2) && pr.scal[5] == 0.0) return;
    block_sum_n<kInitFinThreads, kTerms>(v, red);
    if (threadIdx.x == 0) {
        if (!energy_only) {
            double rz = 0.0, bb = 0.0;        // the workgroups' sums in workgroup order
            for (int w = 0; w < nparts; ++w) {
                rz += pr.scal[kInitPart + 2 * w];
                bb += pr.scal[kInitPart + 2 * w + 1];
            }
            pr.scal[0] = rz;
            pr.scal[1] = rz == 0.0 ? 1.0 : 0.0;
            pr.cg[4] = 0.0;        // the solution so far: x_0 = 0 (generation 0)
            pr.cg[5] = bb;
            if ((check_target & 1) && v[0] + v[1] + v[3] + v[4] <= pr.target) {   // x = 0 above, so the step's update is void
                pr.scal[1] = 1.0;
                pr.scal[2] = 1.0;
                pr.scal[3] = double(gn);
            }
        }
        for (int q = 0; q < kTerms; ++q) pr.scal[8 + kTerms * gn + q] = v[q];
        if (check_target & 4) {
            const CAP_GLOBAL double *e0 = pr.scal.g() + 8 + kTerms * slot_prev;
            const double E0 = e0[0] + e0[1] + e0[3] + e0[4], E1 = v[0] + v[1] + v[3] + v[4];
            reject = !(E1 < E0);
            pr.scal[4] = E1;
            pr.scal[5] = reject ? 1.0 : 0.0;
            pr.scal[6] = E0;
            if (reject) {      // the linearisation (and any stop) at the prediction no longer applies
                pr.scal[1] = 0.0;
                pr.scal[2] = 0.0;
                pr.scal[3] = double(gn_iters);
            }
        }
    }
    if (check_target & 4) {
        __syncthreads();
        if (reject)
            for (int i = threadIdx.x; i < 12 * T.nn; i += blockDim.x) pr.state[i] = pr.state0[i];
    }
}

// Gather A p from the tile partials (no PCG update).
__global__ __launch_bounds__(kNodeThreads) void k_node_gather(const ProbDev *__restrict__ P) {
    const ProbDev &pr = P[blockIdx.x];
    const TemplateDev &T = pr.T;
    const int nn = T.nn;
    for (int i = threadIdx.x; i < 6 * nn; i += blockDim.x) {
        const int c = i / nn, k = i - c * nn;
        pr.Ap[i] = gather_node(T, pr.partial, T.nslots, k, c);
    }
}

// After the last product of a Gauss-Newton step (n = pcg_iters launches of
// k_cg): the last iteration's scalars from the tile sums of launch n - 1, then
// x_n = x_{n-1} + alpha (u_{n-1} + beta p_{n-2}) (or the x at which the
// iteration stopped) and the node update R <- Exp(dw) R, t <- t + dt.  A solve
// stopped at its target energy is left as it is.  Grid: (node blocks, problems).
__global__ __launch_bounds__(256) void k_cg_finish(const ProbDev *__restrict__ P, int n) {
    const ProbDev &pr = P[blockIdx.y];
    const TemplateDev &T = pr.T;
    const int nn = T.nn, nt = T.ntiles, lv = threadIdx.x;
    if (int(blockIdx.x) * 256 >= nn) return;
    if (pr.scal[2] != 0.0) return;                  // stopped at the target energy: no update
    const int k = blockIdx.x * 256 + lv;
    const int gl = (n - 1) & 1;
    double ts[3] = {0.0, 0.0, 0.0};
    const bool stopped = n == 0 || pr.scal[1] != 0.0;
    if (!stopped) {
        wave_sum_n<3>(pr.dots.g() + size_t(gl) * 3 * nt, nt, nt, ts);
    }
    double xu[6], xo[6], po[6];
    if (k < nn) {
        const int xb = stopped ? (n == 0 ? 0 : int(pr.cg[4]) & 1) : gl;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            xo[c] = pr.vx[xb][size_t(c) * nn + k];
            xu[c] = pr.vu[gl][size_t(c) * nn + k];
            po[c] = n >= 2 ? pr.vp[n & 1][size_t(c) * nn + k] : 0.0;
        }
    }
    bool step = false;
    double alpha = 0.0, beta = 0.0;
    if (!stopped) {
        const double gamma = n == 1 ? pr.scal[0] : ts[0], delta = ts[1];
        const double bb = pr.cg[5], rho = n == 1 ? bb : ts[2];
        double den = delta;
        if (n >= 2) {
            const CAP_GLOBAL double *cg = pr.cg.g() + 2 * gl;
            beta = gamma / cg[0];
            den = delta - beta * gamma / cg[1];
        }
        step = !(den <= 0.0 || gamma == 0.0 || (pr.pcg_tol2 > 0.0 && rho <= pr.pcg_tol2 * bb));
        if (step) alpha = gamma / den;
    }
    if (k >= nn) return;
    float x[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        if (step) {
            const double pn = n >= 2 ? fma(beta, po[c], xu[c]) : xu[c];
            x[c] = float(fma(alpha, pn, xo[c]));
        } else {
            x[c] = float(xo[c]);
        }
    }
    node_update_from(pr, k, x, x + 3);
}

// The standard arrangement's node step after product launch j (k_cg with
// kCgStandard): alpha_j = r_j.u_j / p_j.Ap_j (p.Ap from the tile sums, r.u
// from the node blocks of step j - 1), then per node x_{j+1} = x_j + alpha p_j,
// r_{j+1} = r_j - alpha A p_j, u_{j+1} = M r_{j+1}, with the block's r.u and
// r.r for the next product launch; stops (x stays x_j) if p.Ap <= 0.  `last`:
// the node update R <- Exp(dw) R, t <- t + dt from the final x follows.  Grid:
// (node blocks of 256, problems); one thread per node.
__global__ __launch_bounds__(256) void k_pcg_node(const ProbDev *__restrict__ P, int j, int last) {
    __shared__ double red[256 / 64][2];
    const ProbDev &pr = P[blockIdx.y];
    const TemplateDev &T = pr.T;
    const int nn = T.nn, nt = T.ntiles, nb = (nn + 255) / 256, lv = threadIdx.x;
    if (int(blockIdx.x) >= nb) return;
    const int k = blockIdx.x * 256 + lv, kc = min(k, nn - 1);
    // every load up front: the flags, the sums, the node's vectors and partials
    const double target_stop = pr.scal[2], pcg_stopped = pr.scal[1];
    double pap1[1], rz1[1];
    wave_sum_n<1>(pr.dots.g() + nt, nt, nt, pap1);
    wave_sum_n<1>(pr.nsum.g() + size_t((j + 1) & 1) * 2 * nb, nb, nb, rz1);   // (j - 1) & 1; unused at j = 0
    const double pap = pap1[0], rz = j == 0 ? pr.scal[0] : rz1[0];
    const int pb = T.node_pbeg[kc], pe = T.node_pbeg[kc + 1], qmax = max(pe - 1, 0);
    double xo[6], ro[6], po[6];
    float di[6], part[6][kParts];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const size_t o = size_t(c) * nn + kc;
        xo[c] = pr.vx[j & 1][o];
        ro[c] = pr.vr[j & 1][o];
        po[c] = pr.vp[j & 1][o];
        di[c] = pr.dinv[o];
#pragma unroll
        for (int q = 0; q < kParts; ++q) part[c][q] = pr.partial[size_t(c) * T.nslots + min(pb + q, qmax)];
    }
    if (target_stop != 0.0) return;          // stopped at the target energy: no update
    float xn[6];
    if (pcg_stopped != 0.0) {                // stopped earlier: only the final node update
        if (last && k < nn) {
            const int xb = int(pr.cg[4]) & 1;
#pragma unroll
            for (int c = 0; c < 6; ++c) xn[c] = float(pr.vx[xb][size_t(c) * nn + k]);
            node_update_from(pr, k, xn, xn + 3);
        }
        return;
    }
    if (pap <= 0.0) {                        // x stays x_j
        if (blockIdx.x == 0 && lv == 0) {
            pr.scal[1] = 1.0;
            pr.cg[4] = double(j);
        }
        if (last && k < nn) {
#pragma unroll
            for (int c = 0; c < 6; ++c) xn[c] = float(xo[c]);
            node_update_from(pr, k, xn, xn + 3);
        }
        return;
    }
    const double alpha = rz / pap;
    double g = 0.0, r2 = 0.0;
    if (k < nn) {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            float ap = 0.0f;               // A p_j of the node: its partials in order
#pragma unroll
            for (int q = 0; q < kParts; ++q)
                if (pb + q < pe) ap += part[c][q];
            for (int q = pb + kParts; q < pe; ++q) ap += pr.partial[size_t(c) * T.nslots + q];
            const size_t o = size_t(c) * nn + k;
            const double x1 = fma(alpha, po[c], xo[c]);
            const double r1 = fma(-alpha, double(ap), ro[c]);
            const double u1 = double(float(double(di[c]) * r1));   // float32, as multiplied
            xn[c] = float(x1);
            if (!last) {
                pr.vx[(j + 1) & 1][o] = x1;
                pr.vr[(j + 1) & 1][o] = r1;
                pr.vu[(j + 1) & 1][o] = u1;
                g += r1 * u1;
                r2 += r1 * r1;
            }
        }
    }
    if (last) {
        if (k < nn) node_update_from(pr, k, xn, xn + 3);
        return;
    }
    double s2[2] = {g, r2};
    block_sum_n<256, 2>(s2, red);
    if (lv == 0) {
        CAP_GLOBAL double *np = pr.nsum.g() + size_t(j & 1) * 2 * nb;
        np[blockIdx.x] = s2[0];
        np[nb + blockIdx.x] = s2[1];
        if (blockIdx.x == 0) pr.cg[2 * (j & 1)] = rz;
    }
}

}  // namespace cap
