// One trajectory of the tensor jump method, executed by one workgroup.
//
// Paper map (Sec. "Tensor jump method"):
//   traj_init / traj_step        schedule of the sampling MPS, Eqs.
//                                TimeEvolutionFunctions and SimulationStep
//   tdvp                         dynamic TDVP U[dt] (Sec. "Dynamic TDVP"):
//                                1TDVP/2TDVP forward/backward updates,
//                                Lanczos exponentials of effective
//                                Hamiltonians built from cached environments
//   dissipate                    D[tau] = prod_l D_l[tau] (Eq. DissipativeMPO)
//   jump_process                 J_eps (Sec. "Stochastic jump process")
// Decisions that must match any other implementation (switch rule,
// truncation rank, jump / no jump, which jump) are functions of
// gauge-invariant quantities only.
//
// Storage: a site tensor is M[a][s][b] (row-major, current bond dims); a left
// environment at bond b is L[w][a_bra][a_ket]; a right environment at bond b
// is R[w][b_ket][b_bra].  Environments live in numbered slots so that a new
// one can be built while the old one at the same bond is still in use.
#pragma once
#include <dev_gemm.hpp>
#include <dev_linalg.hpp>
#include "tjm_params.h"

template <typename Tc> struct Tjm {
  typedef cplx<Tc> zc;
  const TjmParams& P;
  int* slot;          // LDS [L+2]: env slot of each bond; slot[L+1] is the spare
  int* bA;            // LDS [L+1]: bonds of the sampling MPS
  int* bB;            // LDS [L+1]: bonds of the sampling-layer copy
  // worker scratch
  zc* env; zd* smps; zd* Q; zd* w; zd* v; zc* T1; zd* X; zd* Y; zd* Z; zd* Cb; double* wts;
  zd* oenv; zd* ot;   // MPO observables: two FP64 environments and a stage buffer
  int d, L;

  TJM_DEV Tjm(const TjmParams& p, int* dyn, int worker) : P(p) {
    L = P.L; d = P.d;
    slot = dyn;
    bA = dyn + (L + 2);
    bB = bA + (L + 1);
    char* base = P.scratch + (long)worker * P.scratch_stride;
    env = (zc*)(base + P.off_env);
    smps = (zd*)(base + P.off_smps);
    Q = (zd*)(base + P.off_Q);
    w = (zd*)(base + P.off_w);
    v = (zd*)(base + P.off_v);
    T1 = (zc*)(base + P.off_T1);
    X = (zd*)(base + P.off_X);
    Y = (zd*)(base + P.off_Y);
    Z = (zd*)(base + P.off_Z);
    Cb = (zd*)(base + P.off_C);
    wts = (double*)(base + P.off_wts);
    oenv = (zd*)(base + P.off_oenv);
    ot = (zd*)(base + P.off_ot);
    if (tjm_tid() == 0)                              // environment slot of each bond
      for (int b = 0; b < L + 2; ++b) slot[b] = b;
    tjm_sync();
  }

  TJM_DEV zc* envp(int bond) { return env + (long)slot[bond] * P.env_cap; }
  TJM_DEV zc* spare() { return env + (long)slot[L + 1] * P.env_cap; }
  TJM_DEV void count(int i, unsigned long long n) { if (tjm_tid() == 0) tjm_lds.st[i] += n; }
  TJM_DEV void since(int i, unsigned long long t0) { if (tjm_tid() == 0) tjm_lds.st[i] += tjm_clock() - t0; }
  TJM_DEV static zd* site(zd* mps, const TjmParams& P, int s) { return mps + P.site_off[s]; }

  TJM_DEV unsigned long long mix_nnz(int Dout, int dph, const int* rp) {
    return (unsigned long long)(rp[Dout * dph] - rp[0]);
  }

  // Tile choices of the contractions (tile_mode of the options; the same
  // results under every choice): the effective-Hamiltonian products take
  // wide tiles unless bit 0 is set, the other products only if bit 2 is set;
  // bit 1 selects the small-block variant of the smallest products.
  TJM_DEV int tm_heff() const { return P.tile_mode & 3; }
  TJM_DEV int tm_other() const { return (P.tile_mode & 2) | ((P.tile_mode & 4) ? 0 : 1); }

  // ------------------------------------------------------------------
  // Environments (Fig. TDVP; Sec. "Hybrid strategy")
  // ------------------------------------------------------------------
  TJM_DEV void env_one(zc* e) {
    if (tjm_tid() == 0) e[0] = cmk((Tc)1, (Tc)0);
  }

  // Mixed path: the channel of a new complex-FP32 environment that carries
  // the energy of its half chain (L[en] on the left, R[st] on the right,
  // with en / st the identity channels of the other side) is re-centred on
  // zero, its diagonal mean removed.  FP32 then holds the spread of the
  // Schmidt states' energies instead of an energy of order L, and every
  // effective Hamiltonian built from such environments is H^eff - c I,
  // which multiplies the evolved centre tensor, and so the whole state, by
  // the phase exp(i tau c): observables, norms, Schmidt values and jump
  // probabilities are unchanged.  The shift is exact: the energy channel
  // meets the MPO only through identity blocks that end in the other side's
  // identity channel, so c I in it is c times the identity operator.
  // Skipped at the chain ends, where the single channel is both, and for
  // MPOs without identity channels.
  TJM_DEV void env_center(zc* E, int chi, int chan, int other) {
    if constexpr (sizeof(Tc) == 4) {
      if (chan < 0 || other < 0 || chan == other) return;
      zc* M = E + (long)chan * chi * chi;
      double sum = 0.0;
      for (int a = tjm_tid(); a < chi; a += TJM_NT) sum += (double)M[(long)a * chi + a].re;
      const double mean = blk_sum(sum, tjm_lds.S) / chi;
      for (int a = tjm_tid(); a < chi; a += TJM_NT) M[(long)a * chi + a].re = (Tc)((double)M[(long)a * chi + a].re - mean);
      tjm_sync();
    }
  }

  // L_{s+1}[w'][b'][b] = sum L_s[w][a'][a] conj(A[a'][s'][b']) W[w][w'][s'][s] A[a][s][b]
  TJM_DEVNI void lupdate(int s, const zd* A, int chl, int chr, const zc* Lold, zc* Lnew) {
    const unsigned long long t0 = tjm_clock();
    const int Dl = P.mpoD[s], Dr = P.mpoD[s + 1];
    const int* rp = P.mixL_ptr + (long)s * (P.Dmax * d + 1);
    blk_cgemm_mode<Tc>(tm_other(), chl, d * chr, chl, Dl, false, cmat(Lold, chl, (long)chl * chl), cmat(A, d * chr),
                  T1, d * chr, (long)chl * d * chr, false, tjm_lds.gemm);
    tjm_sync();
    blk_cgemm_mode<Tc>(tm_other(), chr, chr, chl * d, Dr, false, cmat(A, chr, 0, true, true),
                  mix_rows((const zc*)T1, rp, P.mixL, d, (long)chl * d * chr, (long)d * chr, (long)chr),
                  Lnew, chr, (long)chr * chr, false, tjm_lds.gemm);
    tjm_sync();
    env_center(Lnew, chr, P.env_en[s + 1], P.env_st[s + 1]);
    count(TJM_ST_CMAC_MFMA, (unsigned long long)Dl * chl * chl * d * chr + (unsigned long long)Dr * chr * chr * chl * d);
    count(TJM_ST_CMAC_MIX, mix_nnz(Dr, d, rp) * chl * chr);
    since(TJM_ST_T_CONTRACT, t0);
  }

  // R_{s-1}[w][a][a'] = sum B[a][s][b] R_s[w'][b][b'] W[w][w'][s'][s] conj(B[a'][s'][b'])
  // for an MPO block of bonds (Dl, Dr) with mixing rows rp (entries ents),
  // environments and stage buffer Tb in precision TE
  template <typename TE>
  TJM_DEV void env_right(const zd* B, int chl, int chr, int Dl, int Dr, const int* rp, const MixEnt* ents,
                         const cplx<TE>* Rold, cplx<TE>* Rnew, cplx<TE>* Tb) {
    blk_cgemm_mode<TE>(tm_other(), chl * d, chr, chr, Dr, false, cmat(B, chr), cmat(Rold, chr, (long)chr * chr),
                  Tb, chr, (long)chl * d * chr, false, tjm_lds.gemm);
    tjm_sync();
    blk_cgemm_mode<TE>(tm_other(), chl, chl, d * chr, Dl, false,
                  mix_cols((const cplx<TE>*)Tb, rp, ents, d, chr, (long)chl * d * chr, (long)d * chr, (long)chr),
                  cmat(B, d * chr, 0, true, true), Rnew, chl, (long)chl * chl, false, tjm_lds.gemm);
    tjm_sync();
  }

  TJM_DEVNI void rupdate(int s, const zd* B, int chl, int chr, const zc* Rold, zc* Rnew) {
    const unsigned long long t0 = tjm_clock();
    const int Dl = P.mpoD[s], Dr = P.mpoD[s + 1];
    const int* rp = P.mixR_ptr + (long)s * (P.Dmax * d + 1);
    env_right<Tc>(B, chl, chr, Dl, Dr, rp, P.mixR, Rold, Rnew, T1);
    env_center(Rnew, chl, P.env_st[s], P.env_en[s]);
    count(TJM_ST_CMAC_MFMA, (unsigned long long)Dr * chl * d * chr * chr + (unsigned long long)Dl * chl * chl * d * chr);
    count(TJM_ST_CMAC_MIX, mix_nnz(Dl, d, rp) * chl * chr);
    since(TJM_ST_T_CONTRACT, t0);
  }

  // <Psi|O_q|Psi> of MPO observable q on a normalised MPS (Eq. TJMExpVal;
  // Methods, "Resources required for calculating expectation values"): the
  // MPS-MPO-MPS network contracted from the right end with the environment
  // update of TDVP, in FP64 on both paths; the real part
  TJM_DEVNI double mpo_expect(int q, const zd* mps, const int* bd) {
    const int* D = P.oD + (long)q * (L + 1);
    const int rows = P.oDmax * d + 1;
    zd* Ra = oenv;
    zd* Rb = oenv + P.oenv_cap;
    if (tjm_tid() == 0) Ra[0] = cmk(1.0, 0.0);
    tjm_sync();
    for (int s = L - 1; s >= 0; --s) {
      env_right<double>(site((zd*)mps, P, s), bd[s], bd[s + 1], D[s], D[s + 1],
                        P.omixR_ptr + ((long)q * L + s) * rows, P.mixR, Ra, Rb, ot);
      zd* t = Ra; Ra = Rb; Rb = t;
    }
    return gload((const zd*)Ra, 0).re;
  }

  // the MPO observables of a normalised MPS (centre anywhere) into out
  TJM_DEVNI void measure_mpo(const zd* mps, const int* bd, double* out) {
    for (int q = 0; q < P.n_mpo_obs; ++q) {
      const double v = mpo_expect(q, mps, bd);
      if (tjm_tid() == 0) out[P.n_site_obs + q] = v;
    }
  }

  // y[a][s'][c] (+)= sum_s O[s'][s] q[a][s][c] for every (a, c), with DP
  // physical values (d or d^2; d = 2 is the only local dimension); the loads
  // of 8 / DP entries per thread are issued before their stores, and an
  // entry's stores follow its own loads, so y may be q.
  template <int DP>
  TJM_DEV void local_term(const zd* q, zd* y, int chl, int chr, const zd* O, bool acc) {
    constexpr int NE = 8 / DP;
    const int n = chl * chr;
    zd o[DP * DP];
#pragma unroll
    for (int i = 0; i < DP * DP; ++i) o[i] = gload(O, i);
    for (int base = 0; base < n; base += NE * TJM_NT) {
      zd in[NE][DP], yo[NE][DP];
      long off[NE];
#pragma unroll
      for (int u = 0; u < NE; ++u) {
        int e = base + tjm_tid() + u * TJM_NT;
        e = e < n ? e : n - 1;
        const int a = e / chr, c = e - a * chr;
        off[u] = (long)a * DP * chr + c;
#pragma unroll
        for (int s = 0; s < DP; ++s) {
          in[u][s] = gload(q, off[u] + (long)s * chr);
          yo[u][s] = acc ? gload((const zd*)y, off[u] + (long)s * chr) : cmk(0.0, 0.0);
        }
      }
#pragma unroll
      for (int u = 0; u < NE; ++u) {
        if (base + tjm_tid() + u * TJM_NT >= n) continue;
#pragma unroll
        for (int so = 0; so < DP; ++so) {
          zd v = yo[u][so];
#pragma unroll
          for (int s = 0; s < DP; ++s) v = v + o[so * DP + s] * in[u][s];
          gstore(y, off[u] + (long)so * chr, v);
        }
      }
    }
  }

  // ------------------------------------------------------------------
  // Effective Hamiltonians as matrix-free products (Fig. TDVP)
  // ------------------------------------------------------------------
  // Structured products (nearest-neighbour MPO, canonical environments):
  //   y = sum_{b<nL} L[chanL_b] (O_b M) + sum_{b<nR} (O'_b M) R[chanR_b] + Oloc M
  // with M = q[a][s][c] (s < dp), the physical mixings O of each class as
  // CSR rows (see TjmParams), Oloc the local term.  The identity channels
  // of L and R are never read.
  TJM_DEV void heff_struct(const zd* q, zd* y, int chl, int chr, int dp, const zc* Le, const zc* Re,
                           const int* ptrL, const int* ptrR, const int* chanL, const int* chanR, int nL, int nR,
                           const double* loc) {
    const int Dm = P.Dmax;
    const unsigned long long tg = tjm_clock();
    bool acc = false;
    if (nL > 0) {      // left class: (chl x chl) . (chl x dp chr), summed over channels
      blk_cgemm_mode<Tc>(tm_heff(), chl, dp * chr, chl, nL, true, chan_mat(Le, chl, (long)chl * chl, chanL),
                    mix_cols(q, ptrL, P.mixL, dp, chr, 0L, (long)dp * chr, (long)chr), y, dp * chr, 0, false,
                    tjm_lds.gemm);
      tjm_sync();        // the small-product path returns without a barrier
      acc = true;
    }
    if (nR > 0) {      // right class: (chl dp x chr) . (chr x chr), summed over channels
      blk_cgemm_mode<Tc>(tm_heff(), chl * dp, chr, chr, nR, true, mix_rows(q, ptrR, P.mixL, dp, 0L, (long)dp * chr, (long)chr),
                    chan_mat(Re, chr, (long)chr * chr, chanR), y, chr, 0, acc, tjm_lds.gemm);
      tjm_sync();
      acc = true;
    }
    since(TJM_ST_T_GEMM, tg);
    // local term in FP64: y[a][s'][c] += sum_s Oloc[s'][s] q[a][s][c]
    if (dp == 2) local_term<2>(q, y, chl, chr, (const zd*)loc, acc);
    else local_term<4>(q, y, chl, chr, (const zd*)loc, acc);      // dp = d^2
    tjm_sync();
    count(TJM_ST_CMAC_MFMA, (unsigned long long)nL * chl * chl * dp * chr + (unsigned long long)nR * chl * dp * chr * chr);
    count(TJM_ST_CMAC_MIX, (unsigned long long)(ptrL[Dm * dp] - ptrL[0] + ptrR[Dm * dp] - ptrR[0]) * chl * chr);
  }

  struct H1 {            // site s: degree-6 network
    Tjm* t; int s, chl, chr; const zc* Le; const zc* Re;
    TJM_DEVNI void apply(const zd* q, zd* y) {
      const unsigned long long t0 = tjm_clock();
      const TjmParams& P = t->P;
      const int d = t->d, Dl = P.mpoD[s], Dr = P.mpoD[s + 1];
      if (P.structured) {
        const int Dm = P.Dmax;
        const int* rp = P.s1_ptr + (long)s * 2 * (Dm * d + 1);
        t->heff_struct(q, y, chl, chr, d, Le, Re, rp, rp + (Dm * d + 1), P.s1_chan + (long)s * 2 * Dm,
                       P.s1_chan + ((long)s * 2 + 1) * Dm, P.s1_n[2 * s], P.s1_n[2 * s + 1],
                       P.s1_loc + (long)s * d * d * 2);
        t->since(TJM_ST_T_CONTRACT, t0);
        return;
      }
      const int* rp = P.mixL_ptr + (long)s * (P.Dmax * d + 1);
      blk_cgemm_mode<Tc>(t->tm_other(), chl, d * chr, chl, Dl, false, cmat(Le, chl, (long)chl * chl), cmat(q, d * chr),
                    t->T1, d * chr, (long)chl * d * chr, false, tjm_lds.gemm);
      tjm_sync();
      blk_cgemm_mode<Tc>(t->tm_other(), chl * d, chr, chr, Dr, true,
                    mix_rows((const zc*)t->T1, rp, P.mixL, d, (long)chl * d * chr, (long)d * chr, (long)chr),
                    cmat(Re, chr, (long)chr * chr), y, chr, 0, false, tjm_lds.gemm);
      tjm_sync();
      t->count(TJM_ST_CMAC_MFMA, (unsigned long long)Dl * chl * chl * d * chr + (unsigned long long)Dr * chl * d * chr * chr);
      t->count(TJM_ST_CMAC_MIX, t->mix_nnz(Dr, d, rp) * chl * chr);
      t->since(TJM_ST_T_CONTRACT, t0);
    }
  };

  struct H2 {            // sites s, s+1: degree-8 network
    Tjm* t; int s, chl, chr; const zc* Le; const zc* Re;
    TJM_DEVNI void apply(const zd* q, zd* y) {
      const unsigned long long t0 = tjm_clock();
      const TjmParams& P = t->P;
      const int d = t->d, d2 = d * d, Dl = P.mpoD[s], Dr = P.mpoD[s + 2];
      if (P.structured) {
        const int Dm = P.Dmax;
        const int* rp = P.s2_ptr + (long)s * 2 * (Dm * d2 + 1);
        t->heff_struct(q, y, chl, chr, d2, Le, Re, rp, rp + (Dm * d2 + 1), P.s2_chan + (long)s * 2 * Dm,
                       P.s2_chan + ((long)s * 2 + 1) * Dm, P.s2_n[2 * s], P.s2_n[2 * s + 1],
                       P.s2_loc + (long)s * d2 * d2 * 2);
        t->since(TJM_ST_T_CONTRACT, t0);
        return;
      }
      const int* rp = P.mix2_ptr + (long)s * (P.Dmax * d2 + 1);
      blk_cgemm_mode<Tc>(t->tm_other(), chl, d2 * chr, chl, Dl, false, cmat(Le, chl, (long)chl * chl), cmat(q, d2 * chr),
                    t->T1, d2 * chr, (long)chl * d2 * chr, false, tjm_lds.gemm);
      tjm_sync();
      blk_cgemm_mode<Tc>(t->tm_other(), chl * d2, chr, chr, Dr, true,
                    mix_rows((const zc*)t->T1, rp, P.mix2, d2, (long)chl * d2 * chr, (long)d2 * chr, (long)chr),
                    cmat(Re, chr, (long)chr * chr), y, chr, 0, false, tjm_lds.gemm);
      tjm_sync();
      t->count(TJM_ST_CMAC_MFMA, (unsigned long long)Dl * chl * chl * d2 * chr + (unsigned long long)Dr * chl * d2 * chr * chr);
      t->count(TJM_ST_CMAC_MIX, t->mix_nnz(Dr, d2, rp) * chl * chr);
      t->since(TJM_ST_T_CONTRACT, t0);
    }
  };

  struct H0 {            // bond b: degree-4 network, C is kl x kr
    Tjm* t; int b, kl, kr; const zc* Le; const zc* Re;
    TJM_DEVNI void apply(const zd* q, zd* y) {
      const unsigned long long t0 = tjm_clock();
      const TjmParams& P = t->P;
      const int D = P.mpoD[b];
      if (P.structured) {
        // y = C R[st] + L[en] C + sum_{other w} (L[w] C) R[w]
        const int st = P.env_st[b], en = P.env_en[b], nlr = P.lr_n[b];
        const int* lr = P.lr_chan + (long)b * P.Dmax;
        blk_cgemm_mode<Tc>(t->tm_other(), kl, kr, kr, 1, true, cmat(q, kr), cmat(Re + (long)st * kr * kr, kr), y, kr, 0, false,
                      tjm_lds.gemm);
        tjm_sync();      // the small-product path returns without a barrier
        blk_cgemm_mode<Tc>(t->tm_other(), kl, kr, kl, 1, true, cmat(Le + (long)en * kl * kl, kl), cmat(q, kr), y, kr, 0, true,
                      tjm_lds.gemm);
        if (nlr > 0) {
          blk_cgemm_mode<Tc>(t->tm_other(), kl, kr, kl, nlr, false, chan_mat(Le, kl, (long)kl * kl, lr), cmat(q, kr),
                        t->T1, kr, (long)kl * kr, false, tjm_lds.gemm);
          tjm_sync();
          blk_cgemm_mode<Tc>(t->tm_other(), kl, kr, kr, nlr, true, cmat((const zc*)t->T1, kr, (long)kl * kr),
                        chan_mat(Re, kr, (long)kr * kr, lr), y, kr, 0, true, tjm_lds.gemm);
        }
        tjm_sync();
        t->count(TJM_ST_CMAC_MFMA, (unsigned long long)(1 + nlr) * kl * kr * (kl + kr));
        t->since(TJM_ST_T_GEMM, t0);
        t->since(TJM_ST_T_CONTRACT, t0);
        return;
      }
      blk_cgemm_mode<Tc>(t->tm_other(), kl, kr, kl, D, false, cmat(Le, kl, (long)kl * kl), cmat(q, kr),
                    t->T1, kr, (long)kl * kr, false, tjm_lds.gemm);
      tjm_sync();
      blk_cgemm_mode<Tc>(t->tm_other(), kl, kr, kr, D, true, cmat((const zc*)t->T1, kr, (long)kl * kr),
                    cmat(Re, kr, (long)kr * kr), y, kr, 0, false, tjm_lds.gemm);
      tjm_sync();
      t->count(TJM_ST_CMAC_MFMA, (unsigned long long)D * kl * kl * kr + (unsigned long long)D * kl * kr * kr);
      t->since(TJM_ST_T_CONTRACT, t0);
    }
  };

  template <class Op> TJM_DEV void expm(Op& op, zd* vec, int n, double t) {
    const unsigned long long t0 = tjm_clock();
    int it = blk_expm(op, vec, n, t, P.krylov_max, P.krylov_tol, Q, w);
    count(TJM_ST_KRYLOV, (unsigned long long)it);
    count(TJM_ST_EXPM, 1ull);
    since(TJM_ST_T_EXPM, t0);
  }

  // ------------------------------------------------------------------
  // Site moves (FP64 factorisations)
  // ------------------------------------------------------------------
  TJM_DEV void copy(zd* dst, const zd* src, long n) {
    if (n > 0) blk_map((int)n, [&](int e) { return gload(src, e); }, [&](int e, zd x) { gstore(dst, e, x); });
  }

  // next (k x d x c) = C (k x m) . next (m x d x c), via v
  TJM_DEVNI void absorb_right(zd* next, int k, int m, int c) {
    const unsigned long long t0 = tjm_clock();
    blk_cgemm<double>(k, d * c, m, 1, true, cmat((const zd*)Cb, m), cmat((const zd*)next, d * c), v, d * c, 0, false, tjm_lds.gemm);
    tjm_sync();
    copy(next, v, (long)k * d * c);
    tjm_sync();
    since(TJM_ST_T_ABSORB, t0);
  }
  // prev (p x d x k) = prev (p x d x m) . C (m x k), via v
  TJM_DEVNI void absorb_left(zd* prev, int p, int m, int k) {
    const unsigned long long t0 = tjm_clock();
    blk_cgemm<double>(p * d, k, m, 1, true, cmat((const zd*)prev, m), cmat((const zd*)Cb, k), v, k, 0, false, tjm_lds.gemm);
    tjm_sync();
    copy(prev, v, (long)p * d * k);
    tjm_sync();
    since(TJM_ST_T_ABSORB, t0);
  }

  // QR of M_s as (chl d) x chr: M_s <- Q, Cb <- R (k x chr); returns k
  TJM_DEVNI int qr_site(zd* Ms, int chl, int chr) {
    const unsigned long long t0 = tjm_clock();
    const int m = chl * d;
    if (m <= QRF_ROWS && chr <= QRF_COLS) {
      blk_qr_regs(m, chr, Ms, Ms, Cb, Y, false, nullptr);
    } else {
      copy(X, Ms, (long)m * chr);
      tjm_sync();
      blk_qr_global(m, chr, X, Ms, Cb);
    }
    count(TJM_ST_FACT, 1ull);
    since(TJM_ST_T_QR, t0);
    return m < chr ? m : chr;
  }

  // LQ of M_s as chl x (d chr): M_s <- B (k x d chr, orthonormal rows),
  // Cb <- C (chl x k), Z <- C^H (k x chl); returns k
  TJM_DEVNI int lq_site(zd* Ms, int chl, int chr) {
    const unsigned long long t0 = tjm_clock();
    const int n = d * chr;
    const int k = n < chl ? n : chl;
    if (n <= QRF_ROWS && chl <= QRF_COLS) {
      blk_qr_regs(n, chl, Ms, Ms, Cb, Y, true, Z);                  // QR of M^H, written adjoint
    } else {
      for (long e = tjm_tid(); e < (long)n * chl; e += TJM_NT) {    // X = M^H (n x chl)
        int i = (int)(e / chl), j = (int)(e % chl);
        X[e] = conjg(Ms[(long)j * n + i]);
      }
      tjm_sync();
      blk_qr_global(n, chl, X, Y, Z);                               // Y: n x k, Z: k x chl
      for (long e = tjm_tid(); e < (long)k * n; e += TJM_NT) {      // M = Y^H
        int i = (int)(e / n), j = (int)(e % n);
        Ms[e] = conjg(Y[(long)j * k + i]);
      }
      for (long e = tjm_tid(); e < (long)chl * k; e += TJM_NT) {    // C = Z^H
        int i = (int)(e / k), j = (int)(e % k);
        Cb[e] = conjg(Z[(long)j * chl + i]);
      }
      tjm_sync();
    }
    count(TJM_ST_FACT, 1ull);
    since(TJM_ST_T_QR, t0);
    return k;
  }

  TJM_DEVNI void qr_move_right(zd* mps, int* bd, int s) {
    zd* Ms = site(mps, P, s);
    const int chl = bd[s], chr = bd[s + 1], cn = bd[s + 2];
    const int k = qr_site(Ms, chl, chr);
    absorb_right(site(mps, P, s + 1), k, chr, cn);
    if (tjm_tid() == 0) bd[s + 1] = k;
    tjm_sync();
  }

  TJM_DEVNI void lq_move_left(zd* mps, int* bd, int s) {
    zd* Ms = site(mps, P, s);
    const int chl = bd[s], chr = bd[s + 1], cp = bd[s - 1];
    const int k = lq_site(Ms, chl, chr);
    absorb_left(site(mps, P, s - 1), cp, chl, k);
    if (tjm_tid() == 0) bd[s] = k;
    tjm_sync();
  }

  // True if every singular value of the upper-triangular leading n x n block
  // of R (row-major, ld) provably exceeds sqrt(2 thr): sigma_min(R) >=
  // 1 / ||R^{-1}||_F, with R^{-1} by back substitution.  For a wide R
  // [R1 R2], sigma_min >= sigma_min(R1).  Up to 64 columns (every bond of
  // the supported chi_cap) lane c of wavefront 0 builds column c of R^{-1}
  // in LDS, the rows from the bottom in step across the lanes: row i is
  // x_ic = (delta_ic - sum_{j>i} R_ij x_jc) / R_ii for every c at once (x_jc
  // = 0 for j > c comes out of the same formula), so R_ij is one broadcast
  // value per step and x_jc an LDS read of the lane's own column; the sums
  // and the result are those of a per-column substitution.
  TJM_DEVNI bool sv_floor_certified(const zd* R, int n, int ld, double thr) {
    if (n <= 64) {
      zd* X = (zd*)tjm_lds.gemm;                 // X[j][c] = (R^{-1})_{jc}, 64 x 64 complex
      double acc = 0.0;
      int bad = 0;
      if (tjm_wave() == 0) {
        const int c = tjm_lane();
        const bool on = c < n;
        for (int i = n - 1; i >= 0; --i) {
          zd sum = cmk(i == c ? 1.0 : 0.0, 0.0);
          const zd* Ri = R + (long)i * ld;
          for (int j = i + 1; j < n; ++j) sum = sum - Ri[j] * X[j * 64 + c];
          const zd rii = Ri[i];
          const double d2 = abs2(rii);
          if (!(d2 > 0.0)) { bad = 1; break; }   // uniform: every lane reads the same R_ii
          const zd xi = cmk((sum.re * rii.re + sum.im * rii.im) / d2, (sum.im * rii.re - sum.re * rii.im) / d2);
          X[i * 64 + c] = xi;
          if (on) acc += abs2(xi);
        }
      }
      double b2 = (double)bad;
      blk_sum2(acc, b2, tjm_lds.S);
      return b2 == 0.0 && acc * 2.0 * thr < 1.0;
    }
    double acc = 0.0;
    int bad = 0;
    for (int c = tjm_tid(); c < n; c += TJM_NT) {
      zd* x = Y + (long)c * n;
      for (int i = c; i >= 0; --i) {
        zd sum = cmk(i == c ? 1.0 : 0.0, 0.0);
        for (int j = i + 1; j <= c; ++j) sum = sum - R[(long)i * ld + j] * x[j];
        const zd rii = R[(long)i * ld + i];
        const double d2 = abs2(rii);
        if (!(d2 > 0.0)) { bad = 1; break; }
        const zd xi = cmk((sum.re * rii.re + sum.im * rii.im) / d2, (sum.im * rii.re - sum.re * rii.im) / d2);
        x[i] = xi;
        acc += abs2(xi);
      }
    }
    double b2 = (double)bad;
    blk_sum2(acc, b2, tjm_lds.S);
    return b2 == 0.0 && acc * 2.0 * thr < 1.0;
  }

  // Move the centre right with SVD truncation (normalisation sweeps after a
  // jump): M_s = Q R; if R's singular values certifiably all survive the
  // discard threshold the QR move is the result, otherwise R = U S V^H is
  // truncated, M_s = Q U, next <- S V^H next.
  TJM_DEVNI void svd_move_right(zd* mps, int* bd, int s) {
    zd* Ms = site(mps, P, s);
    const int chl = bd[s], chr = bd[s + 1], cn = bd[s + 2];
    const int m = chl * d;
    if (!P.certify) {                                 // SVD of M_s itself
      const unsigned long long ts_ = tjm_clock();
      const int k = blk_svd(m, chr, Ms, Ms, Cb, false, P.svd_discard, P.chi_cap, P.deg_tol, X, Y, Z);
      count(TJM_ST_FACT, 1ull);
      since(TJM_ST_T_SVD, ts_);
      absorb_right(site(mps, P, s + 1), k, chr, cn);
      if (tjm_tid() == 0) bd[s + 1] = k;
      tjm_sync();
      return;
    }
    const int k0 = qr_site(Ms, chl, chr);             // Ms <- Q (m x k0), Cb <- R (k0 x chr)
    const unsigned long long ts_ = tjm_clock();
    const double tot = norm2_site(Cb, (long)k0 * chr);
    int k = k0;
    if (!sv_floor_certified(Cb, k0, chr, P.svd_discard * tot)) {
      k = blk_svd(k0, chr, Cb, w, Cb, false, P.svd_discard, P.chi_cap, P.deg_tol, X, Y, Z);
      count(TJM_ST_FACT, 1ull);
      blk_cgemm<double>(m, k, k0, 1, true, cmat((const zd*)Ms, k0), cmat((const zd*)w, k), v, k, 0, false, tjm_lds.gemm);
      tjm_sync();
      copy(Ms, v, (long)m * k);
      tjm_sync();
    }
    since(TJM_ST_T_SVD, ts_);
    absorb_right(site(mps, P, s + 1), k, chr, cn);
    if (tjm_tid() == 0) bd[s + 1] = k;
    tjm_sync();
  }

  // Mirror image: M_s = C B (LQ); C's singular values certified, or
  // C = U S V^H truncated, M_s <- V^H B, prev <- prev U S.
  TJM_DEVNI void svd_move_left(zd* mps, int* bd, int s) {
    zd* Ms = site(mps, P, s);
    const int chl = bd[s], chr = bd[s + 1], cp = bd[s - 1];
    const int n = d * chr;
    if (!P.certify) {                                 // SVD of M_s itself
      const unsigned long long ts_ = tjm_clock();
      const int k = blk_svd(chl, n, Ms, Cb, Ms, true, P.svd_discard, P.chi_cap, P.deg_tol, X, Y, Z);
      count(TJM_ST_FACT, 1ull);
      since(TJM_ST_T_SVD, ts_);
      absorb_left(site(mps, P, s - 1), cp, chl, k);
      if (tjm_tid() == 0) bd[s] = k;
      tjm_sync();
      return;
    }
    const int k0 = lq_site(Ms, chl, chr);             // Ms <- B (k0 x n), Cb <- C (chl x k0), Z <- C^H
    const unsigned long long ts_ = tjm_clock();
    const double tot = norm2_site(Cb, (long)chl * k0);
    int k = k0;
    if (!sv_floor_certified(Z, k0, chl, P.svd_discard * tot)) {
      k = blk_svd(chl, k0, Cb, Cb, w, true, P.svd_discard, P.chi_cap, P.deg_tol, X, Y, Z);
      count(TJM_ST_FACT, 1ull);
      blk_cgemm<double>(k, n, k0, 1, true, cmat((const zd*)w, k0), cmat((const zd*)Ms, n), v, n, 0, false, tjm_lds.gemm);
      tjm_sync();
      copy(Ms, v, (long)k * n);
      tjm_sync();
    }
    since(TJM_ST_T_SVD, ts_);
    absorb_left(site(mps, P, s - 1), cp, chl, k);
    if (tjm_tid() == 0) bd[s] = k;
    tjm_sync();
  }

  // ------------------------------------------------------------------
  // Dynamic TDVP U[dt] (Sec. "Dynamic TDVP"): an L->R and an R->L
  // half-sweep of tau = dt/2; 2TDVP at bond l iff chi_l < chi_max when the
  // sweep reaches it, else 1TDVP; the turning unit is evolved again.
  // Precondition: centre at site 0, other sites right-canonical.
  // ------------------------------------------------------------------
  TJM_DEVNI void tdvp(zd* mps, int* bd) {
    const double tau = 0.5 * P.dt;
    if (tjm_tid() == 0)
      for (int b = 0; b < L + 2; ++b) slot[b] = b;
    tjm_sync();
    env_one(envp(0));
    env_one(envp(L));
    tjm_sync();
    for (int s = L - 1; s >= 1; --s) {
      rupdate(s, site(mps, P, s), bd[s], bd[s + 1], envp(s + 1), envp(s));
    }
    // left to right
    bool last_two = false;
    for (int s = 0; s < L - 1; ++s) {
      zd* Ms = site(mps, P, s);
      zd* Mn = site(mps, P, s + 1);
      const int chl = bd[s], chm = bd[s + 1], chr = bd[s + 2];
      if (chm < P.chi_max) {
        count(TJM_ST_TWO_SITE, 1ull);
        const unsigned long long tt_ = tjm_clock();
        blk_cgemm<double>(chl * d, d * chr, chm, 1, true, cmat((const zd*)Ms, chm), cmat((const zd*)Mn, d * chr),
                          v, d * chr, 0, false, tjm_lds.gemm);
        tjm_sync();
        since(TJM_ST_T_ABSORB, tt_);
        H2 op{this, s, chl, chr, envp(s), envp(s + 2)};
        expm(op, v, chl * d * d * chr, tau);
        const unsigned long long ts_ = tjm_clock();
    const int k = blk_svd(chl * d, d * chr, v, Ms, Mn, false, P.svd_discard, P.chi_cap, P.deg_tol, X, Y, Z);
        count(TJM_ST_FACT, 1ull);
        since(TJM_ST_T_SVD, ts_);
        if (tjm_tid() == 0) bd[s + 1] = k;
        tjm_sync();
        lupdate(s, Ms, chl, k, envp(s), envp(s + 1));
        if (s + 1 < L - 1) {
          H1 op1{this, s + 1, k, chr, envp(s + 1), envp(s + 2)};
          expm(op1, Mn, k * d * chr, -tau);
        }
        last_two = true;
      } else {
        count(TJM_ST_ONE_SITE, 1ull);
        H1 op{this, s, chl, chm, envp(s), envp(s + 1)};
        expm(op, Ms, chl * d * chm, tau);
        const int k = qr_site(Ms, chl, chm);
        lupdate(s, Ms, chl, k, envp(s), spare());
        H0 op0{this, s + 1, k, chm, spare(), envp(s + 1)};
        expm(op0, Cb, k * chm, -tau);
        if (tjm_tid() == 0) {
          int t = slot[s + 1]; slot[s + 1] = slot[L + 1]; slot[L + 1] = t;
          bd[s + 1] = k;
        }
        tjm_sync();
        absorb_right(Mn, k, chm, chr);
        last_two = false;
      }
    }
    if (L == 1 || !last_two) {
      H1 op{this, L - 1, bd[L - 1], bd[L], envp(L - 1), envp(L)};
      expm(op, site(mps, P, L - 1), bd[L - 1] * d * bd[L], tau);
    }
    // right to left
    last_two = false;
    for (int s = L - 1; s >= 1; --s) {
      zd* Ms = site(mps, P, s);
      zd* Mp = site(mps, P, s - 1);
      const int chp = bd[s - 1], chl = bd[s], chr = bd[s + 1];
      if (chl < P.chi_max) {
        count(TJM_ST_TWO_SITE, 1ull);
        const unsigned long long tt_ = tjm_clock();
        blk_cgemm<double>(chp * d, d * chr, chl, 1, true, cmat((const zd*)Mp, chl), cmat((const zd*)Ms, d * chr),
                          v, d * chr, 0, false, tjm_lds.gemm);
        tjm_sync();
        since(TJM_ST_T_ABSORB, tt_);
        H2 op{this, s - 1, chp, chr, envp(s - 1), envp(s + 1)};
        expm(op, v, chp * d * d * chr, tau);
        const unsigned long long ts_ = tjm_clock();
    const int k = blk_svd(chp * d, d * chr, v, Mp, Ms, true, P.svd_discard, P.chi_cap, P.deg_tol, X, Y, Z);
        count(TJM_ST_FACT, 1ull);
        since(TJM_ST_T_SVD, ts_);
        if (tjm_tid() == 0) bd[s] = k;
        tjm_sync();
        rupdate(s, Ms, k, chr, envp(s + 1), envp(s));
        if (s - 1 > 0) {
          H1 op1{this, s - 1, chp, k, envp(s - 1), envp(s)};
          expm(op1, Mp, chp * d * k, -tau);
        }
        last_two = true;
      } else {
        count(TJM_ST_ONE_SITE, 1ull);
        H1 op{this, s, chl, chr, envp(s), envp(s + 1)};
        expm(op, Ms, chl * d * chr, tau);
        const int k = lq_site(Ms, chl, chr);
        rupdate(s, Ms, k, chr, envp(s + 1), spare());
        H0 op0{this, s, chl, k, envp(s), spare()};
        expm(op0, Cb, chl * k, -tau);
        if (tjm_tid() == 0) {
          int t = slot[s]; slot[s] = slot[L + 1]; slot[L + 1] = t;
          bd[s] = k;
        }
        tjm_sync();
        absorb_left(Mp, chp, chl, k);
        last_two = false;
      }
    }
    if (L == 1 || !last_two) {
      H1 op{this, 0, bd[0], bd[1], envp(0), envp(1)};
      expm(op, site(mps, P, 0), bd[0] * d * bd[1], tau);
    }
  }

  // ------------------------------------------------------------------
  // Dissipative contraction (Eq. DissipativeMPO): M_l <- D_l M_l on the
  // physical index of every site; bond dimensions unchanged.
  // ------------------------------------------------------------------
  TJM_DEVNI void dissipate(zd* mps, const int* bd, const double* Dtab) {
    for (int s = 0; s < L; ++s) {
      zd* M = site(mps, P, s);
      const zd* D = (const zd*)Dtab + (long)s * d * d;
      const int chl = bd[s], chr = bd[s + 1];
      local_term<2>(M, M, chl, chr, D, false);      // M <- D M in place, entry by entry
    }
    tjm_sync();
  }

  // rho[s][s'] = sum_{a,b} M[a][s][b] conj(M[a][s'][b]) at the centre
  // (d = 2): tjm_lds.rho = (rho00, rho11, Re rho01, Im rho01)
  TJM_DEVNI void site_rho(const zd* M, int chl, int chr) {
    double r00 = 0, r11 = 0, rr = 0, ri = 0;
    for (long e = tjm_tid(); e < (long)chl * chr; e += TJM_NT) {
      int a = (int)(e / chr), b = (int)(e % chr);
      zd x0 = M[((long)a * 2 + 0) * chr + b], x1 = M[((long)a * 2 + 1) * chr + b];
      r00 += abs2(x0); r11 += abs2(x1);
      zd c = cdotc(x1, x0);      // x0 conj(x1)
      rr += c.re; ri += c.im;
    }
    blk_sum4(r00, r11, rr, ri, tjm_lds.S);
    if (tjm_tid() == 0) { tjm_lds.rho[0] = r00; tjm_lds.rho[1] = r11; tjm_lds.rho[2] = rr; tjm_lds.rho[3] = ri; }
    tjm_sync();
  }

  // sum_{s,s'} O[s'][s] rho[s][s'] (real part), for a 2x2 operator O
  TJM_DEV double tr_op_rho(const zd* O) {
    zd r01 = cmk(tjm_lds.rho[2], tjm_lds.rho[3]);
    zd v = O[0] * cmk(tjm_lds.rho[0], 0.0) + O[3] * cmk(tjm_lds.rho[1], 0.0) + O[2] * r01 + O[1] * conjg(r01);
    return v.re;
  }

  // Tr(L rho L^dag) for a 2x2 L
  TJM_DEV double tr_l_rho_ld(const zd* Lop) {
    zd rho[4] = {cmk(tjm_lds.rho[0], 0.0), cmk(tjm_lds.rho[2], tjm_lds.rho[3]), cmk(tjm_lds.rho[2], -tjm_lds.rho[3]), cmk(tjm_lds.rho[1], 0.0)};
    double acc = 0.0;
    for (int a = 0; a < 2; ++a) {
      zd x = cmk(0.0, 0.0);
      for (int b = 0; b < 2; ++b)
        for (int c = 0; c < 2; ++c) x = x + Lop[a * 2 + b] * rho[b * 2 + c] * conjg(Lop[a * 2 + c]);
      acc += x.re;
    }
    return acc;
  }

  // measure every observable of site s with the centre at s (rho in tjm_lds.rho)
  TJM_DEV void measure(int s, double* out) {
    if (tjm_tid() == 0) {
      const double tr = tjm_lds.rho[0] + tjm_lds.rho[1];
      for (int q = P.optr[s]; q < P.optr[s + 1]; ++q) {
        int o = P.oidx[q];
        out[o] = tr_op_rho((const zd*)P.obs_op + (long)o * 4) / tr;
      }
    }
  }

  TJM_DEV double norm2_site(const zd* M, long n) {
    double a = 0.0;
    for (long e = tjm_tid(); e < n; e += TJM_NT) a += abs2(M[e]);
    return blk_sum(a, tjm_lds.S);
  }

  TJM_DEV void scale_site(zd* M, long n, double f) {
    for (long e = tjm_tid(); e < n; e += TJM_NT) M[e] = f * M[e];
    tjm_sync();
  }

  // pick the jump from wts (rule of Sec. "Stochastic jump process" with the
  // weights normalised by their sum): first index whose running sum exceeds
  // r W; -1 if W <= 1e-300
  TJM_DEVNI int pick_jump(double r) {
    if (tjm_tid() == 0) {
      double tot = 0.0;
      for (int j = 0; j < P.n_jump; ++j) tot += wts[j];
      int m = -1;
      if (tot > 1e-300) {
        const double thr = r * tot;
        double cum = 0.0;
        for (int j = 0; j < P.n_jump; ++j) {
          cum += wts[j];
          if (cum > thr) { m = j; break; }
        }
        if (m < 0)
          for (int j = P.n_jump - 1; j >= 0; --j)
            if (wts[j] > 0.0) { m = j; break; }
      }
      tjm_lds.pick = m;
    }
    tjm_sync();
    return tjm_lds.pick;
  }

  // apply jump m at its site (centre there), normalise, then the
  // normalisation sweeps through successive SVDs: site -> right end -> 0
  TJM_DEVNI void apply_jump(zd* mps, int* bd, int m, double* obs_out) {
    const int sj = P.jump_site[m];
    zd* M = site(mps, P, sj);
    const zd* Op = (const zd*)P.jump_op + (long)m * 4;
    const int chl = bd[sj], chr = bd[sj + 1];
    for (long e = tjm_tid(); e < (long)chl * chr; e += TJM_NT) {
      int a = (int)(e / chr), b = (int)(e % chr);
      zd in0 = M[((long)a * 2 + 0) * chr + b], in1 = M[((long)a * 2 + 1) * chr + b];
      M[((long)a * 2 + 0) * chr + b] = Op[0] * in0 + Op[1] * in1;
      M[((long)a * 2 + 1) * chr + b] = Op[2] * in0 + Op[3] * in1;
    }
    tjm_sync();
    const long n = (long)chl * d * chr;
    const double nn = norm2_site(M, n);
    scale_site(M, n, 1.0 / sqrt(nn));
    count(TJM_ST_JUMPS, 1ull);
    for (int s = sj; s < L - 1; ++s) svd_move_right(mps, bd, s);
    for (int s = L - 1; s >= 1; --s) {
      if (obs_out) { site_rho(site(mps, P, s), bd[s], bd[s + 1]); measure(s, obs_out); }
      svd_move_left(mps, bd, s);
    }
    finish(mps, bd, obs_out);
  }

  // ------------------------------------------------------------------
  // Jump process J_eps (Sec. "Stochastic jump process") applied to D[tau]
  // of the MPS.  Entry: centre at site 0, the other sites right-canonical.
  // Exit: normalised, centre at site 0, other sites right-canonical.  If
  // obs_out is non-null, the site observables of the resulting state are
  // written there (measured at each centre of the final sweep).
  // Returns the applied jump index, -1 for none, -2 on a non-finite norm.
  // ------------------------------------------------------------------
  TJM_DEVNI int jump_process(zd* mps, int* bd, const double* Dtab, uint32_t step, uint32_t branch,
                             double* obs_out) {
    dissipate(mps, bd, Dtab);
    return jump_sweeps(mps, bd, step, branch, obs_out);
  }

  // The jump process proper, entry after D: QR sweep to the right end for
  // delta p = 1 - ||M_L||^2; no jump (eps >= delta p): normalise and LQ
  // sweep back; otherwise LQ sweep back with the weights at every centre,
  // pick, QR moves to the jump site, apply and normalise through the SVD
  // sweeps.
  TJM_DEVNI int jump_sweeps(zd* mps, int* bd, uint32_t step, uint32_t branch, double* obs_out) {
    for (int s = 0; s < L - 1; ++s) qr_move_right(mps, bd, s);
    const long nlast = (long)bd[L - 1] * d * bd[L];
    const double nrm2 = norm2_site(site(mps, P, L - 1), nlast);
    if (!(nrm2 == nrm2) || nrm2 > 1e300) return -2;
    const double dp = nrm2 < 1.0 ? 1.0 - nrm2 : 0.0;
    double eps, r;
    tjm_draws(P.seed, P.traj_base + (uint32_t)traj_id, step, branch, eps, r);
    if (eps >= dp) {                                  // no jump: normalise
      for (int s = L - 1; s >= 1; --s) {
        if (obs_out) { site_rho(site(mps, P, s), bd[s], bd[s + 1]); measure(s, obs_out); }
        lq_move_left(mps, bd, s);
      }
      finish(mps, bd, obs_out);
      return -1;
    }
    // jump probabilities: sweep the centre right to left
    for (int s = L - 1; s >= 0; --s) {
      site_rho(site(mps, P, s), bd[s], bd[s + 1]);
      if (tjm_tid() == 0) {
        for (int q = P.jptr[s]; q < P.jptr[s + 1]; ++q) {
          int j = P.jidx[q];
          wts[j] = P.jump_rate[j] * tr_l_rho_ld((const zd*)P.jump_op + (long)j * 4);
        }
      }
      if (obs_out) measure(s, obs_out);
      if (s > 0) lq_move_left(mps, bd, s);
    }
    const int m = pick_jump(r);
    if (m < 0) {
      finish(mps, bd, nullptr);
      return -1;
    }
    const int sj = P.jump_site[m];
    for (int s = 0; s < sj; ++s) qr_move_right(mps, bd, s);
    apply_jump(mps, bd, m, obs_out);
    return m;
  }

  // centre at site 0: measure it and normalise
  TJM_DEVNI void finish(zd* mps, int* bd, double* obs_out) {
    zd* M0 = site(mps, P, 0);
    const long n = (long)bd[0] * d * bd[1];
    if (obs_out) { site_rho(M0, bd[0], bd[1]); measure(0, obs_out); }
    const double nn = norm2_site(M0, n);
    scale_site(M0, n, 1.0 / sqrt(nn));
  }

  int traj_id;
  unsigned long long t_begin;

  // ------------------------------------------------------------------
  // Schedule (Eqs. TimeEvolutionFunctions, SimulationStep)
  // ------------------------------------------------------------------
  TJM_DEV void load_bonds(int* bd, const int* src) {
    for (int b = tjm_tid(); b <= L; b += TJM_NT) bd[b] = src[b];
    tjm_sync();
  }
  TJM_DEV void store_bonds(int* dst, const int* bd) {
    for (int b = tjm_tid(); b <= L; b += TJM_NT) dst[b] = bd[b];
    tjm_sync();
  }
  TJM_DEV void stats_begin() {
    for (int i = tjm_tid(); i < TJM_NSTAT; i += TJM_NT) tjm_lds.st[i] = 0ull;
    tjm_sync();
    if (tjm_tid() == 0) t_begin = tjm_clock();
    tjm_sync();
  }
  TJM_DEV void stats_end(int traj) {
    tjm_sync();
    if (tjm_tid() == 0) tjm_lds.st[TJM_ST_T_TOTAL] += tjm_clock() - t_begin;
    tjm_sync();
    for (int i = tjm_tid(); i < TJM_NSTAT; i += TJM_NT) P.tstats[(long)traj * TJM_NSTAT + i] += tjm_lds.st[i];
  }

  // Psi(0): product state, canonicalised; t = 0 observables; Phi = F_0 Psi(0)
  TJM_DEVNI void traj_init(int traj) {
    traj_id = traj;
    stats_begin();
    zd* mps = (zd*)P.mps + (long)traj * P.mps_cap;
    double* o0 = P.obs + (long)traj * (P.n_steps + 1) * P.n_obs;
    if (P.init_mps) {
      // a general MPS: right-canonical from the right end and normalised
      // (centre at site 0); the t = 0 observables come from a copy whose
      // centre is swept back to the right
      for (int b = tjm_tid(); b <= L; b += TJM_NT) bA[b] = P.init_bonds[b];
      tjm_sync();
      for (int s = 0; s < L; ++s)
        copy(site(mps, P, s), site((zd*)P.init_tensors, P, s), (long)bA[s] * d * bA[s + 1]);
      tjm_sync();
      for (int s = L - 1; s >= 1; --s) lq_move_left(mps, bA, s);
      finish(mps, bA, nullptr);
      for (int s = 0; s < L; ++s) copy(site(smps, P, s), site(mps, P, s), (long)bA[s] * d * bA[s + 1]);
      for (int b = tjm_tid(); b <= L; b += TJM_NT) bB[b] = bA[b];
      tjm_sync();
      for (int s = 0; s < L; ++s) {
        site_rho(site(smps, P, s), bB[s], bB[s + 1]);
        measure(s, o0);
        if (s + 1 < L) qr_move_right(smps, bB, s);
      }
    } else {
      // a product state: bonds 1, measured while its centre is swept left
      for (int b = tjm_tid(); b <= L; b += TJM_NT) bA[b] = 1;
      for (long e = tjm_tid(); e < (long)L * d; e += TJM_NT) {
        int s = (int)(e / d), q = (int)(e % d);
        site(mps, P, s)[q] = ((const zd*)P.init_sites)[e];
      }
      tjm_sync();
      for (int s = L - 1; s >= 1; --s) {
        site_rho(site(mps, P, s), bA[s], bA[s + 1]);
        measure(s, o0);
        lq_move_left(mps, bA, s);
      }
      finish(mps, bA, o0);
    }
    if (P.n_mpo_obs) measure_mpo(mps, bA, o0);       // Psi(0), normalised
    int m = -1;                                      // first-order splitting: no F_0
    if (P.order == 2) m = jump_process(mps, bA, P.Dhalf, 0u, 0u, nullptr);
    if (tjm_tid() == 0) {
      P.jlog[(long)traj * 2 * P.n_steps] = m;
      if (m == -2) P.tflags[traj] = 1;
    }
    store_bonds(P.bonds + (long)traj * (L + 1), bA);
    stats_end(traj);
  }

  // F_k for k = 1..n: X = U Phi; Psi_k = J D[dt/2] X (measured);
  // Phi = J D[dt] X for k < n
  TJM_DEVNI void traj_step(int traj, int k) {
    traj_id = traj;
    stats_begin();
    if (P.tflags[traj]) {            // already non-finite: no further work
      stats_end(traj);
      return;
    }
    zd* mps = (zd*)P.mps + (long)traj * P.mps_cap;
    load_bonds(bA, P.bonds + (long)traj * (L + 1));
    tdvp(mps, bA);
    if (P.record_bonds) store_bonds(P.blog + ((long)traj * P.n_steps + (k - 1)) * (L + 1), bA);
    if (P.order == 1) {
      // first-order splitting: Phi = J D[dt] U Phi, measured on its result
      double* o1 = P.obs + ((long)traj * (P.n_steps + 1) + k) * P.n_obs;
      const unsigned long long tj = tjm_clock();
      const int m1 = jump_process(mps, bA, P.Dfull, (uint32_t)k, 0u, o1);
      if (P.n_mpo_obs && m1 != -2) measure_mpo(mps, bA, o1);
      since(TJM_ST_T_JUMP, tj);
      if (tjm_tid() == 0) {
        int* jl = P.jlog + (long)traj * 2 * P.n_steps;
        jl[2 * k - 1] = m1;
        if (k < P.n_steps) jl[2 * k] = -1;
        if (m1 == -2) P.tflags[traj] = 1;
      }
      store_bonds(P.bonds + (long)traj * (L + 1), bA);
      stats_end(traj);
      return;
    }
    for (int s = 0; s < L; ++s) copy(site(smps, P, s), site(mps, P, s), (long)bA[s] * d * bA[s + 1]);
    for (int b = tjm_tid(); b <= L; b += TJM_NT) bB[b] = bA[b];
    tjm_sync();
    double* ok = P.obs + ((long)traj * (P.n_steps + 1) + k) * P.n_obs;
    const unsigned long long tj = tjm_clock();
    int ms = jump_process(smps, bB, P.Dhalf, (uint32_t)k, 1u, ok);
    if (P.n_mpo_obs && ms != -2) measure_mpo(smps, bB, ok);
    int mm = -1;
    if (k < P.n_steps && ms != -2) mm = jump_process(mps, bA, P.Dfull, (uint32_t)k, 0u, nullptr);
    since(TJM_ST_T_JUMP, tj);
    if (tjm_tid() == 0) {
      int* jl = P.jlog + (long)traj * 2 * P.n_steps;
      jl[2 * k - 1] = ms;
      if (k < P.n_steps) jl[2 * k] = mm;
      if (ms == -2 || mm == -2) P.tflags[traj] = 1;
    }
    store_bonds(P.bonds + (long)traj * (L + 1), bA);
    stats_end(traj);
  }
};
