// Per-thread bodies of the reverse pass (adjoint) of the BR D&C eigenvalue
// solver: L = sum_k w_k lambda_k is differentiated back through every merge
// (top-down) and the leaves into dL/dd and dL/de.
//
// Per merge, in reverse order of the forward steps:
//  - assembly (a permutation): gather the parent's adjoints onto the roots,
//    the rotated-away columns and the negligible-z columns;
//  - secular roots and boundary rows, by implicit differentiation of
//    f(lambda) = 1 + rho sum_j z_j^2/(D_j - lambda) = 0.  With
//    a_jk = 1/(D_j - lambda_k), N_k^2 = sum_j z_j^2 a_jk^2, y_k = z o a_k / N_k:
//      dlambda_k/dD_j = z_j^2 a_jk^2 / N_k^2, dlambda_k/dz_j = -2 z_j a_jk / N_k^2,
//      dlambda_k/drho = 1/(rho^2 N_k^2),
//    and blo_k = r_lo . y_k, bhi_k = r_hi . y_k.  Two all-pairs sweeps: one per
//    root (six sums) and one per pole (eight sums);
//  - close-pole rotations, reversed run by run through c, s and t = hypot;
//  - the merge-path sort (a permutation) back onto the children's spectra
//    and boundary rows; the tear coupling collects 2 sign(beta) dL/drho~.
// Leaves: with Q the leaf's eigenvectors, the adjoint of the leaf matrix is
//   Q (diag(gl) + B) Q^T,  B_jk = (q_0j gblo_k + q_{l-1,j} gbhi_k)/(l_k - l_j), j != k,
// and the tear edits d' = d - |beta| send -sign(beta) dL/dd' to each coupling.
// The derivatives are those of the computed (deflated) map, which is the
// method's own.
#pragma once
#include "tde_device.h"

namespace tde {


// Gather the parent's adjoints onto the three lists (mirror of body_assemble).
template <bool Wide>
TDE_DEV void body_bwd_unassemble(long long t, int m, const MergeRec* __restrict__ mr, const Work& w,
                                 const Grad& gr) {
    const MergeRec R = mr[m];
    const int s = R.nL + R.nR;
    const int i = (int)(t - R.pk);
    const long long ks = w.scan[R.pk];
    const int K = (int)(w.scan[R.pk + s] - ks);
    const long long rs = w.scanR[R.pk];
    const int nr = (int)(w.scanR[R.pk + s] - rs);
    const long long ns = R.pk - ks - rs;
    const int nn = s - K - nr;
    const double* Da = w.Da + ks;
    const int* og = w.org + ks;
    const double* ta = w.tau + ks;
    const double* Dr = w.Dr + rs;
    const double* Dd = w.Dd + ns;
    const bool root = (R.flags & MF_ROOT) != 0;
    int pos, list, q;
    if (i < K) {
        const double val = Da[og[i]] + ta[i];
        pos = i + count_lt<Wide>(Dr, nr, val) + count_lt<Wide>(Dd, nn, val);
        list = 0;
        q = i;
    } else if (i < K + nr) {
        q = i - K;
        const double val = Dr[q];
        pos = q + roots_cmp_count<Wide>(Da, og, ta, K, val) + count_lt<Wide>(Dd, nn, val);
        list = 1;
    } else {
        q = i - K - nr;
        const double val = Dd[q];
        pos = q + roots_cmp_count<Wide>(Da, og, ta, K, val) + count_le<Wide>(Dr, nr, val);
        list = 2;
    }
    const long long P = R.off + pos;
    const double gl = gr.glam[P];
    const double gb = root ? 0.0 : gr.gblo[P];
    const double gh = root ? 0.0 : gr.gbhi[P];
    if (list == 0) {
        gr.glr[ks + q] = gl;
        gr.gbr[ks + q] = gb;
        gr.ghr[ks + q] = gh;
    } else if (list == 1) {
        const long long tp = w.rpos[rs + q];
        gr.gD2[tp] = gl;
        gr.gZ2[tp] = 0.0;
        gr.gRL2[tp] = gb;
        gr.gRH2[tp] = gh;
    } else {
        const long long tp = w.dpos[ns + q];
        gr.gD[tp] = gl;
        gr.gZ[tp] = 0.0;
        gr.gRL[tp] = gb;
        gr.gRH[tp] = gh;
    }
}

// Per-root coefficients (first sweep), for root k with origin pole o.
// u_i = zh_i a_ik, a_ik = 1/(D_i - lambda_k) rebuilt from the compact root
// (D_i - D_org) - tau.  The origin term u_o = zh_o/(-tau) is kept out of every
// sum: S = sum_{i != o} u_i^2 is the complement of the origin's weight in
// N^2 = S + u_o^2, which gives the (root, origin) pair's contributions
// without the cancellation that the plain chain rule suffers when z_o is
// small and tau ~ rho z_o^2 (then a_o ~ 1/z_o^2).  coef receives
//   [0..3] gblo/N, gbhi/N, c/N^2, gtot/N^2  (for every pole other than o)
//   [4..7] the root's contributions to its origin pole's dL/dz, dL/dD,
//          dL/drl, dL/drh;
//   [8..9] blo/N, bhi/N (the node's rows, for the dropped couplings).
template <class Red>
TDE_DEV void bwd_root_coeffs(int K, const double* __restrict__ D, const double* __restrict__ zh,
                             const double* __restrict__ RL, const double* __restrict__ RH, int org, double tau,
                             double glam, double gblo, double gbhi, int sub, int G, double* coef) {
    const double Do = D[org];
    double S = 0.0, XL = 0.0, XH = 0.0, A1 = 0.0, A2 = 0.0, A3 = 0.0;
    _Pragma("unroll 2") for (int i = sub; i < K; i += G) {
        const double a = 1.0 / ((D[i] - Do) - tau);
        const double u = (i == org) ? 0.0 : zh[i] * a;
        const double ua = u * a;
        S += u * u;
        XL += RL[i] * u;
        XH += RH[i] * u;
        A1 += RL[i] * ua;
        A2 += RH[i] * ua;
        A3 += u * ua;
    }
    S = Red::sum(S);
    XL = Red::sum(XL);
    XH = Red::sum(XH);
    A1 = Red::sum(A1);
    A2 = Red::sum(A2);
    A3 = Red::sum(A3);
    const double ao = 1.0 / (-tau);
    const double zo = zh[org], rlo = RL[org], rho_ = RH[org];
    const double uo = zo * ao;
    const double N2 = S + uo * uo;
    const double N = sqrt(N2);
    const double blo = (XL + rlo * uo) / N, bhi = (XH + rho_ * uo) / N;
    const double c = gblo * blo + gbhi * bhi;
    // dL/du_o without cancellation: (gb.r_o S - gb.X u_o) / N^3
    const double gbro = gblo * rlo + gbhi * rho_;
    const double gbX = gblo * XL + gbhi * XH;
    const double guo = (gbro * S - gbX * uo) / (N2 * N);
    // gl + sum_{i != o} dL/du_i z_i a_i^2
    const double part = glam + (gblo * A1 + gbhi * A2) / N - c * A3 / N2;
    const double gtot = part + guo * zo * ao * ao;
    const double yo = uo / N;
    coef[0] = gblo / N;
    coef[1] = gbhi / N;
    coef[2] = c / N2;
    coef[3] = gtot / N2;
    coef[4] = guo * ao * ((S - uo * uo) / N2) - 2.0 * zo * ao * part / N2;  // dL/dz_o
    coef[5] = -zo * ao * ao * guo * (S / N2) + yo * yo * part;              // dL/dD_o
    coef[6] = gblo * yo;                                                     // dL/drl_o
    coef[7] = gbhi * yo;                                                     // dL/drh_o
    coef[8] = blo / N;
    coef[9] = bhi / N;
}

// Couplings that deflation drops.  A deflated column p (eigenvector e_p of
// the node) is coupled to the secular eigenvectors y_b by an entry the
// deflated matrix sets to zero: rho z_p z_i for a negligible z_p, and
// E = c s (D_cur - D_nx) between the two columns of a rotated close pair.
// The eigenvalues do not see these entries at first order, but the boundary
// rows do, so the adjoint takes dL/dA_pi + dL/dA_ip for them from the
// eigenvector VJP of the node: with X_p(b) = gblo_p blo_b + gbhi_p bhi_b -
// gblo_b rl_p - gbhi_b rh_p,
//   dL/dA_pi (sym) = z_i sum_b X_p(b) a_pb a_ib / N_b   (secular column i)
// and for the negligible z_p, summed against rho z_i over all i,
//   dL/dz_p = -sum_b X_p(b) a_pb / N_b.
// S receives sum_b {blo_b, bhi_b, gblo_b, gbhi_b}/N_b * a_pb * (a_ib or 1).
template <class Red>
TDE_DEV void bwd_defl_sums(int K, const double* __restrict__ D, const int* __restrict__ org,
                           const double* __restrict__ tau, const double* __restrict__ coef, long long cstride,
                           double Dp, int i, int sub, int G, double* S) {
    const double* gl = coef;
    const double* gh = coef + cstride;
    const double* bl = coef + 8 * cstride;
    const double* bh = coef + 9 * cstride;
    const double Di = (i >= 0) ? D[i] : 0.0;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int b = sub; b < K; b += G) {
        const double Do = D[org[b]];
        double k = rcp_nr((Dp - Do) - tau[b]);
        if (i >= 0) k *= rcp_nr((Di - Do) - tau[b]);
        s0 += bl[b] * k;
        s1 += bh[b] * k;
        s2 += gl[b] * k;
        s3 += gh[b] * k;
    }
    S[0] = Red::sum(s0);
    S[1] = Red::sum(s1);
    S[2] = Red::sum(s2);
    S[3] = Red::sum(s3);
}

// dL/dz of a negligible column (pole Dp, rows rl, rh, row adjoints gbl, gbh).
template <class Red>
TDE_DEV double bwd_negligible_z(int K, const double* __restrict__ D, const int* __restrict__ org,
                                const double* __restrict__ tau, const double* __restrict__ coef, long long cstride,
                                double Dp, double rl, double rh, double gbl, double gbh, int sub, int G) {
    double S[4];
    bwd_defl_sums<Red>(K, D, org, tau, coef, cstride, Dp, -1, sub, G, S);
    return -(gbl * S[0] + gbh * S[1] - rl * S[2] - rh * S[3]);
}

// Per-pole adjoints (second sweep) for active pole j: dL/dz_j, dL/dD_j,
// dL/drl_j, dL/drh_j (post-rotation values).  al, be, ga, mu are views of
// coefficient planes 0..3 (global or staged); corg points at the merge's
// coefficients in the global planes (stride cstride) for the origin terms.
// Roots whose origin is j are skipped in the sums and contribute their
// precomputed origin terms instead (only roots j-1 and j can have origin j).
template <class Red>
TDE_DEV void bwd_pole(int j, int K, const double* __restrict__ D, const int* __restrict__ org,
                      const double* __restrict__ tau, const double* __restrict__ al, const double* __restrict__ be,
                      const double* __restrict__ ga, const double* __restrict__ mu,
                      const double* __restrict__ corg, long long cstride, double zj, double rlj, double rhj,
                      int sub, int G, double* out) {
    const double Dj = D[j];
    double B1 = 0.0, B2 = 0.0, B3 = 0.0, B4 = 0.0, B5 = 0.0, B6 = 0.0, B7 = 0.0, B8 = 0.0;
    _Pragma("unroll 2") for (int k = sub; k < K; k += G) {
        const int ok = org[k];
        const double a = (ok == j) ? 0.0 : 1.0 / ((Dj - D[ok]) - tau[k]);
        const double a2 = a * a;
        B1 += al[k] * a;
        B2 += be[k] * a;
        B3 += ga[k] * a2;
        B4 += mu[k] * a;
        B5 += al[k] * a2;
        B6 += be[k] * a2;
        B7 += ga[k] * a2 * a;
        B8 += mu[k] * a2;
    }
    B1 = Red::sum(B1);
    B2 = Red::sum(B2);
    B3 = Red::sum(B3);
    B4 = Red::sum(B4);
    B5 = Red::sum(B5);
    B6 = Red::sum(B6);
    B7 = Red::sum(B7);
    B8 = Red::sum(B8);
    double gz = rlj * B1 + rhj * B2 - zj * B3 - 2.0 * zj * B4;
    double gD = -zj * (rlj * B5 + rhj * B6 - zj * B7) + zj * zj * B8;
    double grl = zj * B1;
    double grh = zj * B2;
    for (int k = j - 1; k <= j; ++k) {
        if (k < 0 || k >= K || org[k] != j) continue;
        gz += corg[4 * cstride + k];
        gD += corg[5 * cstride + k];
        grl += corg[6 * cstride + k];
        grh += corg[7 * cstride + k];
    }
    out[0] = gz;
    out[1] = gD;
    out[2] = grl;
    out[3] = grh;
}

// Reverse of one rotated pair of a run (see run_step): given the adjoints of
// the deflated column (gdef; its z is a constant 0) and of the survivor (gsv),
// the adjoints of the running column before the step (gc) and of the next
// candidate's unrotated values (gn).  gE is dL/dE for the dropped coupling
// E = c s (D_cur - D_nx) of the pair.  The clamps are not differentiated.
TDE_DEV void run_step_adjoint(const RunState& cur, const RunState& nx, const RunState& gdef, const RunState& gsv,
                              double gE, RunState* gc, RunState* gn) {
    const double t = hypot(cur.Z, nx.Z);
    const double c = nx.Z / t, s = cur.Z / t;
    const double dd = cur.D - nx.D;
    const double gcc = 2.0 * c * cur.D * gdef.D + 2.0 * c * nx.D * gsv.D + cur.L * gdef.L + nx.L * gsv.L +
                       cur.H * gdef.H + nx.H * gsv.H + s * dd * gE;
    const double gss = 2.0 * s * nx.D * gdef.D + 2.0 * s * cur.D * gsv.D - nx.L * gdef.L + cur.L * gsv.L -
                       nx.H * gdef.H + cur.H * gsv.H + c * dd * gE;
    gc->D = c * c * gdef.D + s * s * gsv.D + c * s * gE;
    gn->D = s * s * gdef.D + c * c * gsv.D - c * s * gE;
    gc->L = c * gdef.L + s * gsv.L;
    gn->L = -s * gdef.L + c * gsv.L;
    gc->H = c * gdef.H + s * gsv.H;
    gn->H = -s * gdef.H + c * gsv.H;
    // t = hypot(zc, zn), c = zn/t, s = zc/t
    gc->Z = gsv.Z * s + gcc * (-c * s / t) + gss * (c * c / t);
    gn->Z = gsv.Z * c + gcc * (s * s / t) + gss * (-c * s / t);
}

// Reverse of the close-pole runs: each candidate outside every run copies its
// adjoint through; each run's owner recomputes its chain (same run_step as the
// forward), undoes the run-local sort of the rotated-away columns (the forward
// sorts them by pole value into the run's rotated positions; the same stable
// insertion sort on (value, index) pairs gives the permutation), and walks the
// chain backward.  The adjoint of every column of the run in its unsorted
// order is parked in gD/gZ/gRL/gRH at its own position first: step j reads the
// parked value at candidate j-1 and writes the final adjoint of candidate j,
// whose parked value step j+1 has already consumed.
//
// Dropped couplings: the pair rotated at step j leaves E_j between its
// deflated column and the survivor sv_j, and sv_j = c' def' + s' sv' under
// each later rotation of the same segment, so dL/dE_j sums the node's
// coupling adjoints of def_j with the later deflated columns and with the
// segment's final survivor i (a secular column; one sweep over the roots).
// Two deflated columns at exactly equal poles contribute nothing (the node's
// eigenvectors there are free to rotate and the loss cannot depend on it).
//
// A group of G lanes handles one run: every lane walks the chain (writing the
// same values to the same addresses) and the group splits each O(K) coupling
// sum (lane `sub` of G).
//
// bwd_run_head is the per-candidate first step, one lane per candidate: a
// candidate in no run passes its adjoints straight through (the forward
// copied it), and the candidate that starts a run reports itself so that a
// group can take the run.
TDE_DEV bool bwd_run_head(long long g, int m, const MergeRec* __restrict__ mr, const Work& w, const Grad& gr) {
    const long long t = w.nnpos[g];
    const MergeRec R = mr[m];
    const int s = R.nL + R.nR;
    const long long gs = w.scanC[R.pk], ge = w.scanC[R.pk + s];
    const double tol = merge_tol(w.D, R.pk, s);
    const bool cl_next = (g + 1 < ge) && cand_close(w, g, g + 1, tol);
    const bool cl_prev = (g > gs) && cand_close(w, g - 1, g, tol);
    if (cl_prev) return false;
    if (cl_next) return true;
    gr.gD[t] = gr.gD2[t];
    gr.gZ[t] = gr.gZ2[t];
    gr.gRL[t] = gr.gRL2[t];
    gr.gRH[t] = gr.gRH2[t];
    return false;
}

template <class Red>
TDE_DEV void body_bwd_runs(long long g, int m, const MergeRec* __restrict__ mr, const Work& w, const Grad& gr,
                           long long cstride, int sub, int G) {
    const int* __restrict__ nnpos = w.nnpos;
    const long long t = nnpos[g];
    const MergeRec R = mr[m];
    const int s = R.nL + R.nR;
    const long long gs = w.scanC[R.pk], ge = w.scanC[R.pk + s];
    const double tol = merge_tol(w.D, R.pk, s);
    const bool cl_next = (g + 1 < ge) && cand_close(w, g, g + 1, tol);
    const bool cl_prev = (g > gs) && cand_close(w, g - 1, g, tol);
    if (cl_prev) return;
    if (!cl_next) {
        gr.gD[t] = gr.gD2[t];
        gr.gZ[t] = gr.gZ2[t];
        gr.gRL[t] = gr.gRL2[t];
        gr.gRH[t] = gr.gRH2[t];
        return;
    }
    long long r = g + 1;
    while (r + 1 < ge && cand_close(w, r, r + 1, tol)) ++r;
    RunState cur{w.D[t], w.Z[t], w.RL[t], w.RH[t]};
    for (long long j = g + 1; j <= r; ++j) {
        const long long pj = nnpos[j];
        const RunState nx{w.D[pj], w.Z[pj], w.RL[pj], w.RH[pj]};
        gr.chain[j] = cur;
        RunState def;
        double c, sn;
        if (run_step(&cur, nx, tol, &def, &c, &sn)) {
            gr.cdef[j - 1] = def;
            gr.skey[j - 1] = def.D;
            gr.sidx[j - 1] = (int)(j - 1);
        } else {
            cur = nx;
        }
    }
    for (long long j = g; j < r; ++j) {
        if (w.st[nnpos[j]] != 2) continue;
        const double key = gr.skey[j];
        const int id = gr.sidx[j];
        long long h = j;
        for (long long q = j - 1; q >= g; --q) {
            if (w.st[nnpos[q]] != 2) continue;
            if (gr.skey[q] <= key) break;
            gr.skey[h] = gr.skey[q];
            gr.sidx[h] = gr.sidx[q];
            h = q;
        }
        gr.skey[h] = key;
        gr.sidx[h] = id;
    }
    for (long long q = g; q < r; ++q) {
        const long long pq = nnpos[q];
        const long long po = (w.st[pq] == 2) ? nnpos[gr.sidx[q]] : pq;
        gr.gD[po] = gr.gD2[pq];
        gr.gZ[po] = gr.gZ2[pq];
        gr.gRL[po] = gr.gRL2[pq];
        gr.gRH[po] = gr.gRH2[pq];
    }
    // dL/dE_j for every rotated step j, parked in skey[j - 1] (free again).
    const long long ks = w.scan[R.pk];
    const int K = (int)(w.scan[R.pk + s] - ks);
    const bool rows = (R.flags & MF_ROOT) == 0;
    for (long long j = g + 1; j <= r; ++j) {
        const long long pp = nnpos[j - 1];
        if (w.st[pp] != 2) continue;
        double gE = 0.0;
        if (rows) {
            const RunState dj = gr.cdef[j - 1];
            const double gbl = gr.gRL[pp], gbh = gr.gRH[pp];
            double coefv = 1.0;
            long long q = j + 1;
            for (; q <= r; ++q) {
                const long long pq = nnpos[q - 1];
                if (w.st[pq] != 2) break;
                const RunState cq = gr.chain[q];
                const long long pn = nnpos[q];
                const double tq = hypot(cq.Z, w.Z[pn]);
                const double cc = w.Z[pn] / tq, ss = cq.Z / tq;
                const RunState dq = gr.cdef[q - 1];
                const double den = dq.D - dj.D;
                if (den != 0.0) {
                    const double num = (gr.gRL[pq] * dj.L + gr.gRH[pq] * dj.H) - (gbl * dq.L + gbh * dq.H);
                    gE += coefv * cc * (num / den);
                }
                coefv *= ss;
            }
            // segment survivor: the column written at candidate q - 1
            const long long ps = nnpos[q - 1];
            const int i = (int)(w.scan[ps] - ks);
            double S[4];
            bwd_defl_sums<Red>(K, w.Da + ks, w.org + ks, w.tau + ks, gr.coef + ks, cstride, dj.D, i, sub, G, S);
            const double a2 = w.zhat[ks + i] * (gbl * S[0] + gbh * S[1] - dj.L * S[2] - dj.H * S[3]);
            gE += coefv * a2;
        }
        gr.skey[j - 1] = gE;
    }
    const long long pr = nnpos[r];
    RunState gS{gr.gD2[pr], gr.gZ2[pr], gr.gRL2[pr], gr.gRH2[pr]};
    for (long long j = r; j > g; --j) {
        const long long pj = nnpos[j], pp = nnpos[j - 1];
        const RunState nx{w.D[pj], w.Z[pj], w.RL[pj], w.RH[pj]};
        const RunState prev = gr.chain[j];
        const RunState gout{gr.gD[pp], gr.gZ[pp], gr.gRL[pp], gr.gRH[pp]};
        if (w.st[pp] == 2) {
            RunState gc, gn;
            run_step_adjoint(prev, nx, gout, gS, gr.skey[j - 1], &gc, &gn);
            gr.gD[pj] = gn.D;
            gr.gZ[pj] = gn.Z;
            gr.gRL[pj] = gn.L;
            gr.gRH[pj] = gn.H;
            gS = gc;
        } else {
            gr.gD[pj] = gS.D;
            gr.gZ[pj] = gS.Z;
            gr.gRL[pj] = gS.L;
            gr.gRH[pj] = gS.H;
            gS = gout;
        }
    }
    gr.gD[t] = gS.D;
    gr.gZ[t] = gS.Z;
    gr.gRL[t] = gS.L;
    gr.gRH[t] = gS.H;
}

// Reverse of the merge-path sort and z/row construction: merged position t
// back onto child column src[t] (in place: the children's adjoints overwrite
// the parent's over the same column range).
TDE_DEV void body_bwd_merge(long long t, int m, const MergeRec* __restrict__ mr, const double* __restrict__ e,
                            const unsigned long long* __restrict__ pmax, const Work& w, const Grad& gr) {
    const MergeRec R = mr[m];
    double sgn;
    merge_rho(R, e, pmax, &sgn);
    const double rs2 = 0.70710678118654752440;
    const int i = w.src[t];
    const long long P = R.off + i;
    gr.glam[P] = gr.gD[t];
    if (i < R.nL) {
        gr.gbhi[P] = gr.gZ[t] * rs2;
        gr.gblo[P] = gr.gRL[t];
    } else {
        gr.gblo[P] = sgn * gr.gZ[t] * rs2;
        gr.gbhi[P] = gr.gRH[t];
    }
}

// Leaf adjoint, R rows per lane (rows sub, sub + lanes, ... of the leaf,
// `lanes` lanes per leaf).  sd, se: this lane's own copy of the leaf's torn
// diagonal and off-diagonal (stride st); Q, X: the leaf's eigenvector matrix
// and Q (diag(gl) + B), column-major with leading dimension ld >= nl (element
// (r, k) at [k ld + r]), shared by the leaf's lanes.  bwd_leaf_q recomputes
// the QL, tracking the lane's rows of Q (a row index at or past nl only
// writes rows of the ld x ld block that no lane reads), and stores the
// eigenvalues from the lane that holds row 0; after a barrier body_bwd_leaf_x
// forms row r of X; after another barrier body_bwd_leaf_out writes dL/dd'_r
// and the adjoint of the in-leaf coupling r: gT = X Q^T, gd'_r = gT_rr,
// ge_r = gT_{r,r+1} + gT_{r+1,r}.
TDE_DEV void leaf_load(const LeafRec& L, const double* __restrict__ d, const double* __restrict__ e,
                       const unsigned long long* __restrict__ pmax, double* sd, double* se, int st) {
    const double inv = 1.0 / scale_of(pmax[L.prob]);
    const int nl = L.size;
    for (int i = 0; i < nl; ++i) {
        double di = d[L.off + i] * inv;
        if (i == 0 && (L.flags & LF_TEAR_LEFT)) di -= fabs(e[L.off - 1] * inv);
        if (i == nl - 1 && (L.flags & LF_TEAR_RIGHT)) di -= fabs(e[L.off + nl - 1] * inv);
        sd[i * st] = di;
        se[i * st] = (i + 1 < nl) ? e[L.off + i] * inv : 0.0;
    }
}

// R tracked rows, every rotation applied to each.
template <int R>
struct RowsR {
    RowTrack t[R];
    TDE_DEV void chase_begin(int m) {
#pragma unroll
        for (int k = 0; k < R; ++k) t[k].chase_begin(m);
    }
    TDE_DEV void chase_end(int l) {
#pragma unroll
        for (int k = 0; k < R; ++k) t[k].chase_end(l);
    }
    TDE_DEV void rot(int i, double c, double s) {
#pragma unroll
        for (int k = 0; k < R; ++k) t[k].rot(i, c, s);
    }
    TDE_DEV void swap(int i, int k2) {
#pragma unroll
        for (int k = 0; k < R; ++k) t[k].swap(i, k2);
    }
};

template <int R>
TDE_DEV int bwd_leaf_q(const LeafRec& L, int sub, int lanes, const double* __restrict__ d,
                       const double* __restrict__ e, const unsigned long long* __restrict__ pmax, double* sd,
                       double* se, int st, double* Q, int ld, double* lam) {
    const int nl = L.size;
    leaf_load(L, d, e, pmax, sd, se, st);
    RowsR<R> rows;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        rows.t[k].q = Q + sub + k * lanes;
        rows.t[k].st = ld;
        rows.t[k].init(nl, sub + k * lanes);
    }
    unsigned nrot = 0;
    const int status = leaf_ql_core(nl, sd, se, st, rows, &nrot);
    if (sub == 0)
        for (int k = 0; k < nl; ++k) lam[k] = sd[k * st];
    return status;
}

TDE_DEV void body_bwd_leaf_x(const LeafRec& L, int r, const Grad& gr, const double* Q, int ld, const double* lam,
                             double* X) {
    const int nl = L.size;
    for (int k = 0; k < nl; ++k) {
        const double gb = gr.gblo[L.off + k], gh = gr.gbhi[L.off + k];
        double acc = Q[k * ld + r] * gr.glam[L.off + k];
        for (int j = 0; j < nl; ++j) {
            if (j == k) continue;
            const double den = lam[k] - lam[j];
            if (den == 0.0) continue;
            acc += Q[j * ld + r] * (Q[j * ld] * gb + Q[j * ld + nl - 1] * gh) / den;
        }
        X[k * ld + r] = acc;
    }
}

TDE_DEV void body_bwd_leaf_out(const LeafRec& L, int r, const Grad& gr, const double* Q, const double* X, int ld,
                               double* gd, double* ge) {
    const int nl = L.size;
    double dd = 0.0;
    for (int k = 0; k < nl; ++k) dd += X[k * ld + r] * Q[k * ld + r];
    gr.gdp[L.off + r] = dd;
    gd[L.off + r] = dd;
    if (r + 1 < nl) {
        double off = 0.0;
        for (int k = 0; k < nl; ++k) off += X[k * ld + r] * Q[k * ld + r + 1] + X[k * ld + r + 1] * Q[k * ld + r];
        ge[L.off + r] = off;
    }
}

// Tear coupling of merge m: beta = e[c] (scaled), rho~ = 2|beta| and the torn
// diagonal entries d'_c = d_c - |beta|, d'_{c+1} = d_{c+1} - |beta|.  At beta = 0
// the problem decouples and the derivative is 0.
TDE_DEV void body_bwd_tear(const MergeRec& R, double grho, const double* __restrict__ e,
                           const unsigned long long* __restrict__ pmax, const Grad& gr, double* ge) {
    const long long c = R.off + R.nL - 1;
    const double beta = e[c];
    if (beta == 0.0) {
        ge[c] = 0.0;
        return;
    }
    const double sg = (beta < 0.0) ? -1.0 : 1.0;
    ge[c] = sg * (2.0 * grho - gr.gdp[c] - gr.gdp[c + 1]);
    (void)pmax;
}

}  // namespace tde
