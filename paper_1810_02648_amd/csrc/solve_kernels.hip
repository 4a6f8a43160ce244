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
// Matrix-free J^T |B| J p per tile: dV_i = sum_j w_j (w_k x q_j + tau_k),
// f_i = H_i dV_i, node contributions w_j [q_j x f_i; f_i]; regulariser edges
// u = w_k x e_kl + tau_k - tau_l add w_a [e x u; u] to k and w_a [0; -u] to l.
// ----------------------------------------------------------------------------
template <int kSplit>
__global__ __launch_bounds__(kTileThreads) void k_apply(const ProbDev *__restrict__ P, const TileDesc *__restrict__ D) {
    extern __shared__ float lds[];
    __shared__ int lbeg[kMaxTileSlots + 1];
    __shared__ int ldest[kMaxTileSlots];
    const TileDesc d = D[xcd_item(blockIdx.x, gridDim.x)];
    if (d.prob < 0) return;
    const ProbDev &pr = P[d.prob];
    const TemplateDev &T = pr.T;
    const int nv = T.nv, nn = T.nn, ns = d.ns, nown = d.nown;
    // Global reads come in two dependent rounds: indices (vertex codes and
    // contribution positions, slot nodes, run offsets, destinations, owned
    // edges) and then the data they select; the stop flag is tested between.
    // The first round is branch-free: every thread loads at clamped (in-bounds)
    // positions and replaces what lies outside its ranges afterwards, so all
    // of its loads are in flight together.
    static_assert(kMaxTileSlots < kTileThreads, "one thread per slot and run offset");
    const int lv = threadIdx.x, p = d.vb + lv;
    const bool has_v = lv < d.nvt, has_s = lv < ns, has_e = lv < nown * 8;
    const int pv = min(p, nv - 1), ps = min(d.sb + lv, T.nslots - 1), pl = min(d.sb + lv, T.nslots);
    const int po = min(d.ob + (lv >> 3), nn - 1), pe8 = (lv & 7) * nn + po;
    uint8_t code = pr.vcode[pv];
    int cp[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) cp[j] = T.plan_cpos[size_t(j) * nv + pv];
    int snode = T.slot_node[ps];
    const int sdest = T.slot_dest[ps];
    const int lb = T.list_beg[pl];
    int e_so = T.owned_slot[po], e_se = T.owned_eslot[pe8];
    uint32_t e_cp = T.owned_cpos[pe8];
    const int l0 = T.list_beg[d.sb];
    const double pcg_stopped = pr.scal[1];     // read here, tested below
    // the destinations and run offsets are consumed here, unconditionally, so
    // that their loads are not moved into the branches below (behind the rest)
    __asm__ volatile("" ::"v"(sdest), "v"(lb));
    if (!has_v) {
        code = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) cp[j] = 0;
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
        for (int j = 0; j < 4; ++j) w[j] = T.plan_w[size_t(j) * nv + p];
#pragma unroll
        for (int q6 = 0; q6 < 6; ++q6) Hm[q6] = pr.Hm[size_t(q6) * nv + p];
    }
    // LDS: one 80-byte record per slot (R, node position, p: five float4),
    // then contributions [3][NC] (kSplit) or [6][NC]
    float4 *S = reinterpret_cast<float4 *>(lds);
    float *C = lds + kSlotRec * ns;
    if (has_s) {      // R, position and p of the slot's node
        float sv[20];
#pragma unroll
        for (int q = 0; q < 9; ++q) sv[q] = pr.state[size_t(q) * nn + snode];
#pragma unroll
        for (int q = 0; q < 3; ++q) sv[9 + q] = pr.gpos[size_t(q) * nn + snode];
#pragma unroll
        for (int q = 0; q < 6; ++q) sv[12 + q] = pr.p[size_t(q) * nn + snode];
        sv[18] = sv[19] = 0.0f;
#pragma unroll
        for (int q = 0; q < 5; ++q) S[5 * lv + q] = make_float4(sv[4 * q], sv[4 * q + 1], sv[4 * q + 2], sv[4 * q + 3]);
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
    if (has_v) {
        if (act) {
            float q[4][3];
            float dV[3] = {0, 0, 0};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int sl = (packed >> (8 * j)) & 0xff;
                float R[9], g[3], pp[6];
                slot_rec(S, sl, R, g, pp);
                float dd[3] = {v[0] - g[0], v[1] - g[1], v[2] - g[2]};
                rot_apply(R, dd, q[j]);
                float oxq[3];
                cross3(pp, q[j], oxq);
#pragma unroll
                for (int a = 0; a < 3; ++a) dV[a] += w[j] * (oxq[a] + pp[3 + a]);
            }
            f[0] = (Hm[0] * dV[0] + Hm[1] * dV[1]) + Hm[2] * dV[2];
            f[1] = (Hm[1] * dV[0] + Hm[3] * dV[1]) + Hm[4] * dV[2];
            f[2] = (Hm[2] * dV[0] + Hm[4] * dV[1]) + Hm[5] * dV[2];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float qxf[3];
                cross3(q[j], f, qxf);
                float *cj = C + cp[j];
                cj[0] = w[j] * qxf[0]; cj[NC] = w[j] * qxf[1]; cj[2 * NC] = w[j] * qxf[2];
            }
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                w[j] = 0.0f;      // zero contributions in both passes
                for (int q3 = 0; q3 < 3; ++q3) C[q3 * NC + cp[j]] = 0.0f;
            }
        }
    }
    const float wa = pr.w_arap;
    // regulariser edge k -> l: u = w_k x e_kl + tau_k - tau_l; rotational part e x u
    auto edge_u = [&](int so, int se, float ekl[3], float u[3]) {
        float Rk[9], gk[3], pk[6], Rl[9], gl[3], pl[6];
        slot_rec(S, so, Rk, gk, pk);
        slot_rec(S, se, Rl, gl, pl);
        float dd[3] = {gl[0] - gk[0], gl[1] - gk[1], gl[2] - gk[2]};
        rot_apply(Rk, dd, ekl);
        float oxe[3];
        cross3(pk, ekl, oxe);
        u[0] = (oxe[0] + pk[3]) - pl[3]; u[1] = (oxe[1] + pk[4]) - pl[4]; u[2] = (oxe[2] + pk[5]) - pl[5];
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
    if (kSplit) {
        __syncthreads();
        for (int pair = lv; pair < ns * 3; pair += kTileThreads) {
            const int s = pair / 3, comp = pair - s * 3;
            pr.partial[size_t(comp) * T.nslots + ldest[s]] = run_sum(C + comp * NC, lbeg[s], lbeg[s + 1]);
        }
        __syncthreads();
    }
    if (has_v) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float *cj = C2 + cp[j];
            cj[0] = w[j] * f[0]; cj[NC] = w[j] * f[1]; cj[2 * NC] = w[j] * f[2];
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
        const int s = pair / kComps, comp = pair - s * kComps;
        pr.partial[size_t((kSplit ? 3 : 0) + comp) * T.nslots + ldest[s]] = run_sum(C + comp * NC, lbeg[s], lbeg[s + 1]);
    }
}

template __global__ void k_apply<0>(const ProbDev *, const TileDesc *);
template __global__ void k_apply<1>(const ProbDev *, const TileDesc *);

// ----------------------------------------------------------------------------
// Node kernels: one workgroup per problem.
// ----------------------------------------------------------------------------

constexpr int kItems = 8192 / kNodeThreads;   // node kernels: 8192 items (1365 nodes) in registers
constexpr int kInitItems = 16;   // k_node_init (kInitThreads): the same 8192 items, 256 VGPRs per lane

// Sum of partials [pb, pe) of component c (components are rows of `stride`
// floats: the partials are stored component-major, so the parts of
// neighbouring nodes are neighbours in memory) in order; the
// first kParts loads are issued together (a node is touched by a handful of
// tiles), the rest, if any, one after another.
constexpr int kParts = 8;

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

// After a linearisation: b, diag, Jacobi preconditioner, PCG start vectors
// (x = 0, r = b, z = M^-1 r, p = z), r.z, and the energy of GN step `gn`.
// One thread per (component, node) item; every load is issued before the
// stop tests, and r.z and the energy terms share one block reduction.
// check_target bit 0: stop when the energy reaches the target; bit 1: the
// conditional pass (see k_linearize); bit 2: the learned start's selection
// after the linearisation at the prediction: keep the prediction only if
// its energy is below the energy in scal slot `slot_prev` (that of the
// previous frame's state), otherwise undo any stop (the schedule is again
// gn_iters steps) and restore the start state from state0; scal[4] and
// scal[6] receive the two energies, scal[5] the rejection.
__global__ __launch_bounds__(kInitThreads) void k_node_init(const ProbDev *__restrict__ P, int gn, int energy_only,
                                                          int check_target, int slot_prev, int gn_iters) {
    __shared__ double red[kInitThreads / 64][1 + kTerms];
    __shared__ int reject;
    const ProbDev &pr = P[blockIdx.x];
    const TemplateDev &T = pr.T;
    const int nn = T.nn, n6 = 6 * nn;
    double v[1 + kTerms] = {0, 0, 0, 0, 0, 0};   // r.z, then the energy terms
    for (int t = threadIdx.x; t < T.ntiles; t += blockDim.x)
        for (int q = 0; q < kTerms; ++q) v[1 + q] += pr.tile_e[size_t(t) * kTerms + q];
    const bool regs = n6 <= kInitItems * kInitThreads;
    int pb[kInitItems], pe[kInitItems];
    if (!energy_only && regs) {     // unconditional loads at clamped positions, zeroed past the items
#pragma unroll
        for (int j = 0; j < kInitItems; ++j) {
            const int k = min(int(threadIdx.x) + j * kInitThreads, n6 - 1) % nn;
            pb[j] = T.node_pbeg[k]; pe[j] = T.node_pbeg[k + 1];
        }
#pragma unroll
        for (int j = 0; j < kInitItems; ++j)
            if (int(threadIdx.x) + j * kInitThreads >= n6) pb[j] = pe[j] = 0;
    }
    // stopped at the target energy (never so at the selection, which follows
    // the frame set-up's cleared flags)
    if (pr.scal[2] != 0.0 && !(check_target & 4)) return;
    if ((check_target & 2) && pr.scal[5] == 0.0) return;   // conditional pass (see k_linearize)
    if (!energy_only) {
        if (regs) {
            // items in groups of four, each group's loads (b and the diagonal,
            // kParts parts each) in flight together
            constexpr int G = 4;
            static_assert(kInitItems % G == 0, "whole groups");
#pragma unroll
            for (int g = 0; g < kInitItems; g += G) {
                if (g * kInitThreads >= n6) break;           // (uniform) no thread has these items
                int cb[G], cd[G], gb[G], ge[G];
                float bb[G], dd[G];
#pragma unroll
                for (int h = 0; h < G; ++h) {
                    cb[h] = min(int(threadIdx.x) + (g + h) * kInitThreads, n6 - 1) / nn;
                    cd[h] = 6 + cb[h];
                    gb[h] = pb[g + h];
                    ge[h] = pe[g + h];
                }
                sum_parts_n<G>(pr.partial, T.nslots, cb, gb, ge, bb);
                sum_parts_n<G>(pr.partial, T.nslots, cd, gb, ge, dd);
#pragma unroll
                for (int h = 0; h < G; ++h) {
                    const int i = threadIdx.x + (g + h) * kInitThreads;
                    if (i < n6) {
                        const float b = bb[h], d = dd[h];
                        const float mi = d > 0.0f ? 1.0f / d : 1.0f;
                        const float z = mi * b;
                        pr.b[i] = b; pr.diag[i] = d; pr.dinv[i] = mi;
                        pr.x[i] = 0.0f; pr.r[i] = b; pr.z[i] = z; pr.p[i] = z;
                        v[0] += double(b) * double(z);
                    }
                }
            }
        } else {
            for (int i = threadIdx.x; i < n6; i += blockDim.x) {
                const int c = i / nn, k = i - c * nn;
                const float b = gather_node(T, pr.partial, T.nslots, k, c);
                const float d = gather_node(T, pr.partial, T.nslots, k, 6 + c);
                const float mi = d > 0.0f ? 1.0f / d : 1.0f;
                const float z = mi * b;
                pr.b[i] = b; pr.diag[i] = d; pr.dinv[i] = mi;
                pr.x[i] = 0.0f; pr.r[i] = b; pr.z[i] = z; pr.p[i] = z;
                v[0] += double(b) * double(z);
            }
        }
    }
    block_sum_n<kInitThreads, 1 + kTerms>(v, red);
    if (threadIdx.x == 0) {
        const double rz = v[0];
        if (!energy_only) {
            pr.scal[0] = rz;
            pr.scal[1] = rz == 0.0 ? 1.0 : 0.0;
            if ((check_target & 1) && v[1] + v[2] + v[4] + v[5] <= pr.target) {   // x = 0 above, so the step's update is void
                pr.scal[1] = 1.0;
                pr.scal[2] = 1.0;
                pr.scal[3] = double(gn);
            }
        }
        for (int q = 0; q < kTerms; ++q) pr.scal[8 + kTerms * gn + q] = v[1 + q];
        if (check_target & 4) {
            const CAP_GLOBAL double *e0 = pr.scal.g() + 8 + kTerms * slot_prev;
            const double E0 = e0[0] + e0[1] + e0[3] + e0[4], E1 = v[1] + v[2] + v[4] + v[5];
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

// One PCG iteration after k_apply: A p, alpha, x/r/z updates, beta, p.
// Stops (for this GN step) when p.Ap <= 0 or r.z == 0.  `last`: apply the
// node update afterwards; `update_only`: only that.  Items are (component,
// node) pairs; each thread keeps its items' values in registers between phases.
__global__ __launch_bounds__(kNodeThreads) void k_node_pcg(const ProbDev *__restrict__ P, int last, int update_only) {
    __shared__ double red[kNodeThreads / 64];
    const ProbDev &pr = P[blockIdx.x];
    const TemplateDev &T = pr.T;
    const int nn = T.nn, n6 = 6 * nn;
    if (!update_only && n6 <= kItems * kNodeThreads) {
        // every load of the iteration up front (p, x, r, 1/diag, the node's
        // partial range, r.z and the stop flag), then the partial sums
        float pp[kItems], xx[kItems], rr[kItems], di[kItems];
        int pb[kItems], pe[kItems];
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const int i = threadIdx.x + j * kNodeThreads;
            pp[j] = xx[j] = rr[j] = di[j] = 0.0f;
            pb[j] = pe[j] = 0;
            if (i < n6) {
                const int k = i % nn;
                pp[j] = pr.p[i]; xx[j] = pr.x[i]; rr[j] = pr.r[i]; di[j] = pr.dinv[i];
                pb[j] = T.node_pbeg[k]; pe[j] = T.node_pbeg[k + 1];
            }
        }
        const double rz = pr.scal[0];
        if (pr.scal[1] == 0.0) {
            float ap[kItems];
            double pap = 0.0;
#pragma unroll
            for (int j = 0; j < kItems; ++j) {
                const int c = (threadIdx.x + j * kNodeThreads) / nn;
                ap[j] = sum_parts(pr.partial, T.nslots, c, pb[j], pe[j]);
                pap += double(pp[j]) * double(ap[j]);
            }
            pap = block_sum<kNodeThreads>(pap, red);
            if (pap <= 0.0) {
                if (threadIdx.x == 0) pr.scal[1] = 1.0;
            } else {
                const double alpha = rz / pap;
                double rz2 = 0.0;
                float zz[kItems];
#pragma unroll
                for (int j = 0; j < kItems; ++j) {
                    const int i = threadIdx.x + j * kNodeThreads;
                    zz[j] = 0.0f;
                    if (i < n6) {
                        pr.x[i] = float(fma(alpha, double(pp[j]), double(xx[j])));
                        const float r = float(fma(-alpha, double(ap[j]), double(rr[j])));
                        const float z = di[j] * r;
                        pr.r[i] = r;
                        zz[j] = z;
                        rz2 += double(r) * double(z);
                    }
                }
                rz2 = block_sum<kNodeThreads>(rz2, red);
                const double beta = rz2 / rz;
#pragma unroll
                for (int j = 0; j < kItems; ++j) {
                    const int i = threadIdx.x + j * kNodeThreads;
                    if (i < n6) pr.p[i] = float(fma(beta, double(pp[j]), double(zz[j])));
                }
                if (threadIdx.x == 0) {
                    pr.scal[0] = rz2;
                    if (rz2 == 0.0) pr.scal[1] = 1.0;
                }
            }
        }
    } else if (!update_only && pr.scal[1] == 0.0) {      // more items than registers
        double pap = 0.0;
        for (int i = threadIdx.x; i < n6; i += kNodeThreads) {
            const int c = i / nn, k = i - c * nn;
            const float a = gather_node(T, pr.partial, T.nslots, k, c);
            pr.Ap[i] = a;
            pap += double(pr.p[i]) * double(a);
        }
        pap = block_sum<kNodeThreads>(pap, red);
        const double rz = pr.scal[0];
        if (pap <= 0.0) {
            if (threadIdx.x == 0) pr.scal[1] = 1.0;
        } else {
            const double alpha = rz / pap;
            double rz2 = 0.0;
            for (int i = threadIdx.x; i < n6; i += kNodeThreads) {
                pr.x[i] = float(fma(alpha, double(pr.p[i]), double(pr.x[i])));
                const float r = float(fma(-alpha, double(pr.Ap[i]), double(pr.r[i])));
                const float z = pr.dinv[i] * r;
                pr.r[i] = r;
                pr.z[i] = z;
                rz2 += double(r) * double(z);
            }
            rz2 = block_sum<kNodeThreads>(rz2, red);
            const double beta = rz2 / rz;
            for (int i = threadIdx.x; i < n6; i += kNodeThreads) pr.p[i] = float(fma(beta, double(pr.p[i]), double(pr.z[i])));
            if (threadIdx.x == 0) {
                pr.scal[0] = rz2;
                if (rz2 == 0.0) pr.scal[1] = 1.0;
            }
        }
    }
    if (last || update_only) {
        __syncthreads();
        for (int k = threadIdx.x; k < nn; k += blockDim.x) node_update(pr, k);
    }
}

// ----------------------------------------------------------------------------
// PCG iteration for large node counts, split over several workgroups per
// problem (blockIdx.x = item block of kSplitItems (component, node) items).
// Dot products are summed per workgroup, then every workgroup adds the
// workgroup sums in block order, so all of them see the same value.  r.z
// alternates between scal[0] (even iterations) and scal[7] (odd), so the
// workgroup that stores the next value never races a reader of the current.
// ----------------------------------------------------------------------------
__device__ inline int split_blocks(int nn) { return (6 * nn + kSplitItems - 1) / kSplitItems; }

// A p from the tile partials, and the workgroup's share of p.Ap.
__global__ __launch_bounds__(kSplitThreads) void k_pcg_split_a(const ProbDev *__restrict__ P) {
    __shared__ double red[kSplitThreads / 64];
    const ProbDev &pr = P[blockIdx.y];
    const TemplateDev &T = pr.T;
    const int nn = T.nn, n6 = 6 * nn;
    if (pr.scal[1] != 0.0 || int(blockIdx.x) >= split_blocks(nn)) return;
    double pap = 0.0;
    for (int u = 0; u < kSplitItems / kSplitThreads; ++u) {
        const int i = blockIdx.x * kSplitItems + u * kSplitThreads + threadIdx.x;
        if (i < n6) {
            const int c = i / nn, k = i - c * nn;
            const float a = gather_node(T, pr.partial, T.nslots, k, c);
            pr.Ap[i] = a;
            pap += double(pr.p[i]) * double(a);
        }
    }
    pap = block_sum<kSplitThreads>(pap, red);
    if (threadIdx.x == 0) pr.dots[blockIdx.x] = pap;
}

// alpha = r.z / p.Ap; x, r, z updates; the workgroup's share of the new r.z.
__global__ __launch_bounds__(kSplitThreads) void k_pcg_split_b(const ProbDev *__restrict__ P, int it) {
    __shared__ double red[kSplitThreads / 64];
    const ProbDev &pr = P[blockIdx.y];
    const int nn = pr.T.nn, n6 = 6 * nn, G = split_blocks(nn);
    if (pr.scal[1] != 0.0 || int(blockIdx.x) >= G) return;
    double pap = 0.0;
    for (int w = 0; w < G; ++w) pap += pr.dots[w];
    if (pap <= 0.0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) pr.scal[1] = 1.0;
        return;
    }
    const double alpha = pr.scal[(it & 1) ? 7 : 0] / pap;
    double rz2 = 0.0;
    for (int u = 0; u < kSplitItems / kSplitThreads; ++u) {
        const int i = blockIdx.x * kSplitItems + u * kSplitThreads + threadIdx.x;
        if (i < n6) {
            pr.x[i] = float(fma(alpha, double(pr.p[i]), double(pr.x[i])));
            const float r = float(fma(-alpha, double(pr.Ap[i]), double(pr.r[i])));
            const float z = pr.dinv[i] * r;
            pr.r[i] = r;
            pr.z[i] = z;
            rz2 += double(r) * double(z);
        }
    }
    rz2 = block_sum<kSplitThreads>(rz2, red);
    if (threadIdx.x == 0) pr.dots[G + blockIdx.x] = rz2;
}

// beta = r.z' / r.z; p = z + beta p; the next r.z into the other slot.  With
// `last`, the node update follows for this workgroup's share of the nodes.
__global__ __launch_bounds__(kSplitThreads) void k_pcg_split_c(const ProbDev *__restrict__ P, int it, int last) {
    const ProbDev &pr = P[blockIdx.y];
    const int nn = pr.T.nn, n6 = 6 * nn, G = split_blocks(nn);
    if (int(blockIdx.x) >= G) return;
    if (pr.scal[1] == 0.0) {
        double rz2 = 0.0;
        for (int w = 0; w < G; ++w) rz2 += pr.dots[G + w];
        const double beta = rz2 / pr.scal[(it & 1) ? 7 : 0];
        for (int u = 0; u < kSplitItems / kSplitThreads; ++u) {
            const int i = blockIdx.x * kSplitItems + u * kSplitThreads + threadIdx.x;
            if (i < n6) pr.p[i] = float(fma(beta, double(pr.p[i]), double(pr.z[i])));
        }
        __syncthreads();
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            pr.scal[(it & 1) ? 0 : 7] = rz2;
            if (rz2 == 0.0) pr.scal[1] = 1.0;
        }
    }
    if (last) {
        const int per = (nn + G - 1) / G;
        for (int k = blockIdx.x * per + threadIdx.x; k < min(nn, int(blockIdx.x + 1) * per); k += blockDim.x)
            node_update(pr, k);
    }
}

}  // namespace cap
