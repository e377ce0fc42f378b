// kf_kernels.hpp -- single-pass look-back scan kernels for the parallel
// Kalman filter (Algorithm 5), the RTS smoother's reverse scan (Algorithm 6)
// and the two-filter smoother's backward scan fused with the combination
// (Algorithm 7), plus the per-model preparation kernel.
//
// Tiling: one workgroup of BLOCK threads per tile of BLOCK*L time steps; a
// thread owns L consecutive steps.  Per tile:
//   1. load inputs, build the elements, fold each thread's L elements (serial);
//   2. scan the thread aggregates across the workgroup (wavefront Hillis-Steele
//      over lanes, then the per-wave totals through LDS);
//   3. publish the tile aggregate, look back over earlier tiles (windowed,
//      one wavefront), publish the tile's anchored inclusive prefix;
//   4. each thread applies its exclusive prefix to its own steps in order and
//      writes the outputs.
// Tiles are taken in scan order from an atomic counter, so every tile a block
// waits on belongs to a block that is already running.  The status words and
// counters are zeroed by the preparation kernel that precedes the scans.
#pragma once
#include <cstdint>
#include <type_traits>

#include "kf_scan.hpp"

namespace kfs {

// Derived model quantities, FP64-computed once per call (eqs. pkf_init1..3):
//   generic element (k >= 2): S = H Q H^T + R, K = Q H^T S^{-1},
//     A = (I - K H) F, C = (I - K H) Q, W = F^T H^T S^{-1}, J = W H F,
//     b_k = K y_k, eta_k = W y_k;
//   first element (k = 1): x = F m0, P = F P0 F^T + Q, S1 = H P H^T + R,
//     K1 = P H^T S1^{-1}, A_1 = 0, b_1 = c1 + K1 y_1 with c1 = x - K1 H x,
//     C_1 = P - K1 S1 K1^T, eta_1 = W y_1, J_1 = J (reading C4).
// The model itself (F, Q, H, R, m0, P0) is copied for the per-step updates
// and the smoothing elements.  For the time-invariant pipelines, SL is the
// matrix part of an aggregate of L consecutive generic elements and
// PHI[i], PSI[i] (i < L) map y at the i-th step of such an aggregate to its
// vector part:  b = sum_i PHI[i] y_i,  eta = sum_i PSI[i] y_i.
// Layout (type R):
template <int N, int M, int L = 1> struct CL {
  static constexpr int A = 0, C = A + N * N, J = C + N * N, K = J + N * N, W = K + N * M,
                       K1 = W + N * M, c1 = K1 + N * M, C1 = c1 + N, F = C1 + N * N,
                       Q = F + N * N, H = Q + N * N, Rm = H + M * N, m0 = Rm + M * M,
                       P0 = m0 + N, SL = P0 + N * N, PHI = SL + 3 * N * N,
                       PSI = PHI + L * N * M, SIZE = PSI + L * N * M;
};
// A second set of aggregate tables, for the backward two-filter scan's L,
// after the largest first set (kMaxItems steps).
constexpr int kMaxItems = 16;
template <int N, int M, int L> struct CLB {
  static constexpr int SL = CL<N, M, kMaxItems>::SIZE, PHI = SL + 3 * N * N,
                       PSI = PHI + L * N * M, SIZE = PSI + L * N * M;
};

// The preparation launch also zeroes the workspace's control region (tile
// tickets, epochs, timeout flags, look-back status words and payloads) with a
// grid-stride loop.  In block b < nmodels (one block per model of a batch,
// block 0 alone for a shared model), wavefront 0 derives the generic element and
// then the aggregate tables, each doubling step one Lemma 1 combine spread
// over 16 lanes (mpart_combine_lanes), while wavefront 1 derives the first
// element, so the FP64 chains overlap.
//
// Aggregate tables by doubling (L a power of two): with S_h the matrix part of
// h consecutive generic elements and PHI_h[j], PSI_h[j] (j < h) its vector
// coefficients, Lemma 1 for S_h (x) S_h (coefficients P1..P4, see
// mpart_combine_lanes) gives
//   j <  h:  PHI_2h[j] = P1 PHI_h[j],              PSI_2h[j] = PSI_h[j] - P4 PHI_h[j]
//   j >= h:  PHI_2h[j] = P2 PSI_h[j-h] + PHI_h[j-h], PSI_2h[j] = P3 PSI_h[j-h]
// starting from S_1 = (A, C, J), PHI_1[0] = K, PSI_1[0] = W.
template <int N, int M, class R, int L, int LB>
__global__ __launch_bounds__(256) void k_prepare(const R* __restrict__ F_, const R* __restrict__ Q_,
                                                 const R* __restrict__ H_, const R* __restrict__ R_,
                                                 const R* __restrict__ m0_,
                                                 const R* __restrict__ P0_, R* __restrict__ cst,
                                                 unsigned* __restrict__ ctrl, size_t ctrl_words,
                                                 long nmodels, long cst_stride) {
  static_assert((L & (L - 1)) == 0 && (LB & (LB - 1)) == 0 && L <= kMaxItems && LB <= kMaxItems,
                "aggregate lengths must be powers of two up to kMaxItems");
  constexpr int LMAX = L > LB ? L : LB;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < ctrl_words;
       i += (size_t)gridDim.x * blockDim.x)
    ctrl[i] = 0u;
  // block b derives model b (models are packed back to back)
  const long mdl = blockIdx.x;
  if (mdl >= nmodels) return;
  F_ += mdl * N * N;
  Q_ += mdl * N * N;
  H_ += mdl * M * N;
  R_ += mdl * M * M;
  m0_ += mdl * N;
  P0_ += mdl * N * N;
  cst += mdl * cst_stride;
  using D = double;
  using LY = CL<N, M, L>;
  __shared__ MPart<N, D> sS[2];       // S_h, double-buffered
  __shared__ D sPc[4][N][N];          // P1..P4 of S_h (x) S_h
  __shared__ D sW[4][N][N];           // combine scratch
  __shared__ D sPHI[2][LMAX][N][M], sPSI[2][LMAX][N][M];
  const int tid = threadIdx.x, lane = tid & (WAVE - 1);
  // The two elements are derived entry-parallel in FP64, one wavefront each
  // (lane r*cols + c owns entry (r, c) of each product, the wavefront
  // synchronising between products), with the same operations per entry as
  // the sequential formulas; symmetric results are formed from the upper
  // triangle in both lanes (r, c) and (c, r).
  __shared__ D mF[2][N][N], mQ[2][N][N], mH[2][M][N], mR[2][M][M];
  const int l = lane;
  const int wv = tid / WAVE;
  // The model is read with every load issued before the first LDS write, so
  // that the reads take one round trip instead of one per matrix: lanes past
  // a matrix's size read its entry 0 and do not store it.  Wavefront 1 also
  // reads m0 and P0 here.
  D ld_p0 = D(0), ld_m0 = D(0);
  if (wv < 2) {
    const int lf = l < N * N ? l : 0, lh = l < M * N ? l : 0, lr = l < M * M ? l : 0;
    const D f = D(F_[lf]), q = D(Q_[lf]), h = D(H_[lh]), r = D(R_[lr]);
    if (wv == 1) {
      ld_p0 = D(P0_[lf]);
      ld_m0 = D(m0_[l < N ? l : 0]);
    }
    if (l < N * N) {
      mF[wv][l / N][l % N] = f;
      mQ[wv][l / N][l % N] = q;
    }
    if (l < M * N) mH[wv][l / N][l % N] = h;
    if (l < M * M) mR[wv][l / M][l % M] = r;
    wave_lds_sync();
  }
  if (wv == 0) {
    // generic element (eq. pkf_init1)
    const D(&F)[N][N] = mF[0];
    const D(&Q)[N][N] = mQ[0];
    const D(&H)[M][N] = mH[0];
    const D(&Rm)[M][M] = mR[0];
    __shared__ D gHQ[M][N], gHF[M][N], gS[M][M], gKt[M][N], gWt[M][N], gIKH[N][N];
    if (l < M * N) {
      const int i = l / N, j = l % N;
      D hq = D(0), hf = D(0);
#pragma unroll
      for (int t = 0; t < N; ++t) {
        hq += H[i][t] * Q[t][j];
        hf += H[i][t] * F[t][j];
      }
      gHQ[i][j] = hq;
      gHF[i][j] = hf;
    }
    wave_lds_sync();
    if (l < M * M) {  // S = H Q H^T + R
      const int i = l / M, j = l % M, a = i < j ? i : j, b = i < j ? j : i;
      D sv = Rm[a][b];
#pragma unroll
      for (int t = 0; t < N; ++t) sv += gHQ[a][t] * H[b][t];
      gS[i][j] = sv;
    }
    wave_lds_sync();
    if (l < N) {  // column l of K^T = S^{-1} H Q and of W^T = S^{-1} H F
      D Sr[M][M], sd[M], B[M][2];
#pragma unroll
      for (int i = 0; i < M; ++i) {
#pragma unroll
        for (int j = 0; j < M; ++j) Sr[i][j] = gS[i][j];
        B[i][0] = gHQ[i][l];
        B[i][1] = gHF[i][l];
      }
      chol_factor<M, D>(Sr, sd);
      chol_solve<M, 2, D>(Sr, sd, B);
#pragma unroll
      for (int i = 0; i < M; ++i) {
        gKt[i][l] = B[i][0];
        gWt[i][l] = B[i][1];
      }
    }
    wave_lds_sync();
    D Jv = D(0);
    if (l < N * N) {  // I - K H, and J = (S^{-1} H F)^T (H F)
      const int i = l / N, j = l % N, a = i < j ? i : j, b = i < j ? j : i;
      D v = (i == j) ? D(1) : D(0);
#pragma unroll
      for (int t = 0; t < M; ++t) {
        v -= gKt[t][i] * H[t][j];
        Jv += gWt[t][a] * gHF[t][b];
      }
      gIKH[i][j] = v;
    }
    wave_lds_sync();
    if (l < N * N) {  // A = (I - K H) F, C = (I - K H) Q symmetrised
      const int i = l / N, j = l % N;
      D av = D(0), c1 = D(0), c2 = D(0);
#pragma unroll
      for (int t = 0; t < N; ++t) {
        av += gIKH[i][t] * F[t][j];
        c1 += gIKH[i][t] * Q[t][j];
        c2 += gIKH[j][t] * Q[t][i];
      }
      const D Cs = 0.5 * (c1 + c2);
      cst[LY::A + i * N + j] = R(av);
      cst[LY::C + i * N + j] = R(Cs);
      cst[LY::J + i * N + j] = R(Jv);
      sS[0].A[i][j] = av;
      sS[0].C[i][j] = Cs;
      sS[0].J[i][j] = Jv;
    }
    if (l < N * M) {
      const int i = l / M, t = l % M;
      cst[LY::K + i * M + t] = R(gKt[t][i]);
      cst[LY::W + i * M + t] = R(gWt[t][i]);
      sPHI[0][0][i][t] = gKt[t][i];
      sPSI[0][0][i][t] = gWt[t][i];
    }
  } else if (wv == 1) {
    // first element (eq. pkf_init2) and the model copies
    const D(&F)[N][N] = mF[1];
    const D(&Q)[N][N] = mQ[1];
    const D(&H)[M][N] = mH[1];
    const D(&Rm)[M][M] = mR[1];
    __shared__ D fP0[N][N], fm0[N], fx[N], fFP[N][N], fP[N][N], fHP[M][N], fHx[M], fS[M][M],
        fK[M][N];
    if (l < N * N) fP0[l / N][l % N] = ld_p0;
    if (l < N) fm0[l] = ld_m0;
    wave_lds_sync();
    if (l < N * N) {  // copies: F, Q and P0 symmetrised, m0
      const int i = l / N, j = l % N;
      cst[LY::F + l] = R(F[i][j]);
      cst[LY::Q + l] = R(0.5 * (Q[i][j] + Q[j][i]));
      cst[LY::P0 + l] = R(0.5 * (fP0[i][j] + fP0[j][i]));
      D fp = D(0);
#pragma unroll
      for (int t = 0; t < N; ++t) fp += F[i][t] * fP0[t][j];
      fFP[i][j] = fp;
    }
    if (l < N) {
      D xv = D(0);
#pragma unroll
      for (int t = 0; t < N; ++t) xv += F[l][t] * fm0[t];
      fx[l] = xv;
      cst[LY::m0 + l] = R(fm0[l]);
    }
    if (l < M * N) cst[LY::H + l] = R(H[l / N][l % N]);
    if (l < M * M) cst[LY::Rm + l] = R(0.5 * (Rm[l / M][l % M] + Rm[l % M][l / M]));
    wave_lds_sync();
    if (l < N * N) {  // P = F P0 F^T + Q
      const int i = l / N, j = l % N, a = i < j ? i : j, b = i < j ? j : i;
      D pv = Q[a][b];
#pragma unroll
      for (int t = 0; t < N; ++t) pv += fFP[a][t] * F[b][t];
      fP[i][j] = pv;
    }
    wave_lds_sync();
    if (l < M * N) {  // H P
      const int i = l / N, j = l % N;
      D hp = D(0);
#pragma unroll
      for (int t = 0; t < N; ++t) hp += H[i][t] * fP[t][j];
      fHP[i][j] = hp;
    }
    if (l < M) {
      D hx = D(0);
#pragma unroll
      for (int t = 0; t < N; ++t) hx += H[l][t] * fx[t];
      fHx[l] = hx;
    }
    wave_lds_sync();
    if (l < M * M) {  // S1 = H P H^T + R
      const int i = l / M, j = l % M, a = i < j ? i : j, b = i < j ? j : i;
      D sv = Rm[a][b];
#pragma unroll
      for (int t = 0; t < N; ++t) sv += fHP[a][t] * H[b][t];
      fS[i][j] = sv;
    }
    wave_lds_sync();
    if (l < N) {  // column l of K1^T = S1^{-1} H P
      D Sr[M][M], sd[M], B[M][1];
#pragma unroll
      for (int i = 0; i < M; ++i) {
#pragma unroll
        for (int j = 0; j < M; ++j) Sr[i][j] = fS[i][j];
        B[i][0] = fHP[i][l];
      }
      chol_factor<M, D>(Sr, sd);
      chol_solve<M, 1, D>(Sr, sd, B);
#pragma unroll
      for (int i = 0; i < M; ++i) fK[i][l] = B[i][0];
    }
    wave_lds_sync();
    if (l < N) {  // c1 = x - K1 H x
      D cv = fx[l];
#pragma unroll
      for (int t = 0; t < M; ++t) cv -= fK[t][l] * fHx[t];
      cst[LY::c1 + l] = R(cv);
    }
    if (l < N * M) cst[LY::K1 + (l / M) * M + l % M] = R(fK[l % M][l / M]);
    if (l < N * N) {  // C_1 = P - (H P)^T S1^{-1} (H P)
      const int i = l / N, j = l % N, a = i < j ? i : j, b = i < j ? j : i;
      D cv = fP[a][b];
#pragma unroll
      for (int t = 0; t < M; ++t) cv -= fHP[t][a] * fK[t][b];
      cst[LY::C1 + l] = R(cv);
    }
  }
  // doubling, all in wavefront 0 (lanes synchronise among themselves); the
  // tables of h consecutive elements are written out when h reaches L (first
  // set) and LB (second set)
  if (tid >= WAVE) return;
  wave_lds_sync();
  auto write_set = [&](int cur, int h, int sl, int phi, int psi) {
    if (lane < h) {
#pragma unroll
      for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c < M; ++c) {
          cst[phi + lane * N * M + r * M + c] = R(sPHI[cur][lane][r][c]);
          cst[psi + lane * N * M + r * M + c] = R(sPSI[cur][lane][r][c]);
        }
    }
    if (lane < N * N) {
      const int r = lane / N, c = lane % N;
      cst[sl + r * N + c] = R(sS[cur].A[r][c]);
      cst[sl + N * N + r * N + c] = R(sS[cur].C[r][c]);
      cst[sl + 2 * N * N + r * N + c] = R(sS[cur].J[r][c]);
    }
  };
  int cur = 0;
#pragma unroll 1
  for (int h = 1; h < LMAX; h *= 2) {
    mpart_combine_lanes<N, D>(sS[cur], sS[cur], sS[cur ^ 1], sPc, sW, lane);
    const int j = lane;
    if (j < 2 * h) {
      D nphi[N][M], npsi[N][M];
      if (j < h) {
        D T1[N][M];
        mm<N, N, M, D>(sPc[0], sPHI[cur][j], nphi);
        mm<N, N, M, D>(sPc[3], sPHI[cur][j], T1);
#pragma unroll
        for (int r = 0; r < N; ++r)
#pragma unroll
          for (int c = 0; c < M; ++c) npsi[r][c] = sPSI[cur][j][r][c] - T1[r][c];
      } else {
        D T1[N][M];
        mm<N, N, M, D>(sPc[1], sPSI[cur][j - h], T1);
#pragma unroll
        for (int r = 0; r < N; ++r)
#pragma unroll
          for (int c = 0; c < M; ++c) nphi[r][c] = T1[r][c] + sPHI[cur][j - h][r][c];
        mm<N, N, M, D>(sPc[2], sPSI[cur][j - h], npsi);
      }
      copy_mat<N, M, D>(nphi, sPHI[cur ^ 1][j]);
      copy_mat<N, M, D>(npsi, sPSI[cur ^ 1][j]);
    }
    wave_lds_sync();
    cur ^= 1;
    if (2 * h == L) write_set(cur, L, LY::SL, LY::PHI, LY::PSI);
    if (2 * h == LB) write_set(cur, LB, CLB<N, M, LB>::SL, CLB<N, M, LB>::PHI, CLB<N, M, LB>::PSI);
  }
  if (L == 1) write_set(cur, 1, LY::SL, LY::PHI, LY::PSI);
  if (LB == 1) write_set(cur, 1, CLB<N, M, LB>::SL, CLB<N, M, LB>::PHI, CLB<N, M, LB>::PSI);
}

// Output stores are plain (write-back) stores: the L2 merges the 16-byte
// pieces a thread writes for consecutive rows into whole lines before they
// reach memory.  Non-temporal stores would send every piece to memory on its
// own, which costs several times more.
template <class R> KF_DEV void st_out(R* p, R v) { *p = v; }

// Zeroes the workspace's control region (in place of the preparation kernel
// when there are no model constants to derive).
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_clear(unsigned* __restrict__ ctrl, size_t words) {
  for (size_t i = blockIdx.x * (size_t)BLOCK + threadIdx.x; i < words; i += (size_t)gridDim.x * BLOCK)
    ctrl[i] = 0u;
}

// Ragged batches: validate every sequence and lay out the tiles of both scan
// slots, whose tiles hold tile0 and tile1 steps.  start[s][i] is the first
// tile ticket of sequence i (start[s][nseq] the number of tiles), map[s][g]
// the sequence of ticket g, -1 from the last tile up to the grid size bound[s].
// A sequence with fewer than one step or rows outside [0, total_steps) gets no
// tiles; if any sequence is invalid, or the valid lengths add up to more than
// total_steps, bit 1 of both slots' error words is raised (and in the latter
// case no sequence gets tiles), so no kernel ever touches rows outside the
// arrays.  One block.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_batch_tiles(
    const int64_t* __restrict__ len, const int64_t* __restrict__ row, long nseq, long total_steps,
    long tile0, long tile1, int64_t* __restrict__ start0, int64_t* __restrict__ start1,
    int* __restrict__ map0, int* __restrict__ map1, long bound0, long bound1,
    unsigned* __restrict__ err0, unsigned* __restrict__ err1) {
  __shared__ long long s_a[BLOCK], s_b[BLOCK];
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  auto valid = [&](long i) {
    const long T = (long)len[i], r = (long)row[i];
    return T >= 1 && T <= total_steps && r >= 0 && r <= total_steps - T;
  };
  if (tid == 0) s_bad = 0;
  __syncthreads();
  long long part = 0;
  int bad = 0;
  for (long i = tid; i < nseq; i += BLOCK) {
    if (valid(i)) part += (long long)len[i];
    else bad = 1;
  }
  if (bad) atomicOr(&s_bad, 1);
  s_a[tid] = part;
  __syncthreads();
  for (int o = BLOCK / 2; o > 0; o >>= 1) {
    if (tid < o) s_a[tid] += s_a[tid + o];
    __syncthreads();
  }
  const bool over = s_a[0] > (long long)total_steps;
  if (tid == 0 && (s_bad || over)) {
    atomicOr(err0, 2u);
    atomicOr(err1, 2u);
  }
  __syncthreads();
  long long c0 = 0, c1 = 0;
  for (long b = 0; b < nseq; b += BLOCK) {
    const long i = b + tid;
    long long n0 = 0, n1 = 0;
    if (i < nseq && !over && valid(i)) {
      n0 = ((long long)len[i] + tile0 - 1) / tile0;
      n1 = ((long long)len[i] + tile1 - 1) / tile1;
    }
    s_a[tid] = n0;
    s_b[tid] = n1;
    __syncthreads();
    for (int o = 1; o < BLOCK; o <<= 1) {
      const long long x = (tid >= o) ? s_a[tid - o] : 0, y = (tid >= o) ? s_b[tid - o] : 0;
      __syncthreads();
      s_a[tid] += x;
      s_b[tid] += y;
      __syncthreads();
    }
    if (i < nseq) {
      start0[i] = c0 + s_a[tid] - n0;
      start1[i] = c1 + s_b[tid] - n1;
    }
    c0 += s_a[BLOCK - 1];
    c1 += s_b[BLOCK - 1];
    __syncthreads();
  }
  if (tid == 0) {
    start0[nseq] = c0;
    start1[nseq] = c1;
  }
  __threadfence_block();
  __syncthreads();
  for (long i = tid; i < nseq; i += BLOCK) {
    for (long g = (long)start0[i]; g < (long)start0[i + 1]; ++g) map0[g] = (int)i;
    for (long g = (long)start1[i]; g < (long)start1[i + 1]; ++g) map1[g] = (int)i;
  }
  for (long g = (long)c0 + tid; g < bound0; g += BLOCK) map0[g] = -1;
  for (long g = (long)c1 + tid; g < bound1; g += BLOCK) map1[g] = -1;
}

// Look-back state and sizes shared by the scans (array pointers travel as
// separate kernel parameters, see IO below).  agg and pre hold tagged words
// (kf_scan.hpp): kWords<R> per scalar.
template <class R> struct ScanArgs {
  int* flags;      // [nseq * ntiles] status words
  u64* agg;        // [nseq * ntiles][elem size * kWords]
  u64* pre;        // [nseq * ntiles][anchored prefix size * kWords]
  unsigned* ctr;   // [0] tile ticket, [1] finished blocks, [2] look-back timeout flag
  unsigned* epoch; // the epoch of the previous pass (its tag), on a cache line of its own
  long T;
  long ntiles;     // tiles per sequence
  long nseq;
  // ragged batches (all null / zero for equal-length sequences):
  const int* tile_seq;          // [grid] sequence of each tile ticket, -1 past the last tile
  const int64_t* tile_start;    // [nseq + 1] first ticket of each sequence
  const int64_t* seq_len;       // [nseq] steps of each sequence
  const int64_t* seq_row;       // [nseq] first row of each sequence in y and the outputs
  long cst_stride;              // scalars per model in cst when every sequence has its own
};

KF_DEV long uniform(long v) {
  const unsigned long long u = (unsigned long long)v;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
  return (long)(((unsigned long long)hi << 32) | lo);
}

// The sequence a tile belongs to, as bound into a pipeline.
struct SeqInfo {
  long T;        // steps
  long ntiles;   // tiles
  long row0;     // first row in y and the outputs
  long model;    // model index (0 when the model is shared)
};

// The kernels take the array pointers as separate __restrict__ parameters
// (not through ScanArgs): with the no-alias guarantee the compiler keeps
// the uniform model constants in scalar registers (s_load) even after the
// look-back's atomics, and may reorder the streaming loads and stores.
template <class R> struct IO {
  const R* __restrict__ cst;
  const R* __restrict__ y;
  const R* __restrict__ m_in;
  const R* __restrict__ P_in;
  R* __restrict__ m_out;
  R* __restrict__ P_out;
};

// Element of step k (0-based row k, i.e. time step k+1) from its measurement.
template <int N, int M, class R>
KF_DEV FElem<N, R> filter_element(const R* __restrict__ cst, long k, const R (&y)[M]) {
  using L = CL<N, M>;
  FElem<N, R> a;
  const bool first = (k == 0);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    R b = first ? cst[L::c1 + i] : R(0);
    R e = R(0);
#pragma unroll
    for (int t = 0; t < M; ++t) {
      b += (first ? cst[L::K1 + i * M + t] : cst[L::K + i * M + t]) * y[t];
      e += cst[L::W + i * M + t] * y[t];
    }
    a.b[i] = b;
    a.e[i] = e;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      a.A[i][j] = first ? R(0) : cst[L::A + i * N + j];
      a.C[i][j] = first ? cst[L::C1 + i * N + j] : cst[L::C + i * N + j];
      a.J[i][j] = cst[L::J + i * N + j];
    }
  }
  return a;
}

// ---------------------------------------------------------------------------
// Time-varying models (u, d optional).  Row r of the per-step arrays holds
// F_r, Q_r, u_r (the prediction into step r+1) and H_{r+1}, R_{r+1}, d_{r+1};
// m0, P0 are the prior.  Shared by all sequences of a call.
// ---------------------------------------------------------------------------
template <class R> struct TvModel {
  const R* F;
  const R* Q;
  const R* H;
  const R* Rm;
  const R* u;   // may be null (zero)
  const R* d;   // may be null (zero)
  const R* m0;
  const R* P0;
};

template <int N, class R> KF_DEV void load_mat(const R* __restrict__ p, R (&A)[N][N]) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) A[i][j] = p[i * N + j];
}

// Filtering element of row r (step r+1) of a time-varying model: eqs.
// pkf_init1 (r > 0) and pkf_init2 (r = 0) with the inputs u, d, and
// eq. pkf_init3 for (eta, J) (reading C4 at r = 0), factorisations in P::S.
template <int N, int M, class P>
KF_DEV FElem<N, typename P::R> filter_element_tv(const TvModel<typename P::R>& tv, long r,
                                                  const typename P::R (&yk)[M]) {
  using R = typename P::R;
  using S = typename P::S;
  R F[N][N], Q[N][N], H[M][N], Rm[M][M], u[N], d[M];
  load_mat<N, R>(tv.F + r * N * N, F);
  load_mat<N, R>(tv.Q + r * N * N, Q);
#pragma unroll
  for (int i = 0; i < M; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) H[i][j] = tv.H[r * M * N + i * N + j];
#pragma unroll
    for (int j = 0; j < M; ++j) Rm[i][j] = tv.Rm[r * M * M + i * M + j];
    d[i] = tv.d ? tv.d[r * M + i] : R(0);
  }
#pragma unroll
  for (int i = 0; i < N; ++i) u[i] = tv.u ? tv.u[r * N + i] : R(0);
  FElem<N, R> e;
  // S = H Q H^T + R (the S of eq. pkf_init1), residual v = y - H u - d
  S HQ[M][N], Sm[M][M], sd[M];
  mm<M, N, N, S>(H, Q, HQ);
  sym_xyt_plus<M, N, S>(HQ, H, Rm, Sm);
  chol_factor<M, S>(Sm, sd);
  S HF[M][N], B[M][N + 1];  // [S^{-1} H F | S^{-1} v]
  mm<M, N, N, S>(H, F, HF);
#pragma unroll
  for (int i = 0; i < M; ++i) {
    S v = S(yk[i]) - S(d[i]);
#pragma unroll
    for (int t = 0; t < N; ++t) {
      v -= S(H[i][t]) * S(u[t]);
      B[i][t] = HF[i][t];
    }
    B[i][N] = v;
  }
  S vres[M];
#pragma unroll
  for (int i = 0; i < M; ++i) vres[i] = B[i][N];
  chol_solve<M, N + 1, S>(Sm, sd, B);
  // eta = (H F)^T S^{-1} v,  J = (H F)^T S^{-1} (H F)
#pragma unroll
  for (int i = 0; i < N; ++i) {
    S s = S(0);
#pragma unroll
    for (int t = 0; t < M; ++t) s += HF[t][i] * B[t][N];
    e.e[i] = R(s);
  }
  S Jm[N][N], Z[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) Z[i][j] = S(0);
  {
    S SiHF[M][N];
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) SiHF[i][j] = B[i][j];
    sym_xty_plus<N, M, S>(HF, SiHF, Z, Jm);
  }
  copy_mat<N, N, R>(Jm, e.J);
  if (r > 0) {
    S Kt[M][N];  // K^T = S^{-1} H Q
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) Kt[i][j] = HQ[i][j];
    chol_solve<M, N, S>(Sm, sd, Kt);
    S IKH[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) {
        S s = (i == j) ? S(1) : S(0);
#pragma unroll
        for (int t = 0; t < M; ++t) s -= Kt[t][i] * S(H[t][j]);
        IKH[i][j] = s;
      }
    S A[N][N], C[N][N];
    mm<N, N, N, S>(IKH, F, A);
    mm<N, N, N, S>(IKH, Q, C);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      S s = S(u[i]);  // b = u + K v
#pragma unroll
      for (int t = 0; t < M; ++t) s += Kt[t][i] * vres[t];
      e.b[i] = R(s);
#pragma unroll
      for (int j = 0; j < N; ++j) {
        e.A[i][j] = R(A[i][j]);
        e.C[i][j] = R(S(0.5) * (C[i][j] + C[j][i]));
      }
    }
  } else {
    // eq. pkf_init2: predict the prior, then condition on y_1
    R m0[N], P0[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i) m0[i] = tv.m0[i];
    load_mat<N, R>(tv.P0, P0);
    S xp[N], FP[N][N], Pp[N][N];
    mv<N, N, S>(F, m0, xp);
#pragma unroll
    for (int i = 0; i < N; ++i) xp[i] += S(u[i]);
    mm<N, N, N, S>(F, P0, FP);
    sym_xyt_plus<N, N, S>(FP, F, Q, Pp);
    S HP[M][N + 1], S1[M][M], s1d[M];
    {
      S HPm[M][N];
      mm<M, N, N, S>(H, Pp, HPm);
#pragma unroll
      for (int i = 0; i < M; ++i) {
        S v = S(yk[i]) - S(d[i]);
#pragma unroll
        for (int t = 0; t < N; ++t) {
          v -= S(H[i][t]) * xp[t];
          HP[i][t] = HPm[i][t];
        }
        HP[i][N] = v;
      }
      sym_xyt_plus<M, N, S>(HPm, H, Rm, S1);
    }
    chol_factor<M, S>(S1, s1d);
    S K1[M][N + 1];  // [S1^{-1} H Pp | S1^{-1} v1]
#pragma unroll
    for (int i = 0; i < M; ++i)
#pragma unroll
      for (int j = 0; j <= N; ++j) K1[i][j] = HP[i][j];
    chol_solve<M, N + 1, S>(S1, s1d, K1);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      S s = xp[i];
#pragma unroll
      for (int t = 0; t < M; ++t) s += HP[t][i] * K1[t][N];
      e.b[i] = R(s);
#pragma unroll
      for (int j = 0; j < N; ++j) e.A[i][j] = R(0);
    }
    // C_1 = Pp - (H Pp)^T S1^{-1} (H Pp), upper triangle mirrored
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = i; j < N; ++j) {
        S s = Pp[i][j];
#pragma unroll
        for (int t = 0; t < M; ++t) s -= HP[t][i] * K1[t][j];
        e.C[i][j] = R(s);
        e.C[j][i] = R(s);
      }
  }
  return e;
}

// Smoothing element of row k of a time-varying model (eq. prts_init1 with
// F_{k+1}, Q_{k+1}, u_{k+1}: g = x - E (F x + u)); eq. prts_init2 at the last row.
template <int N, class P>
KF_DEV SElem<N, typename P::R> rts_element_tv(const TvModel<typename P::R>& tv, long T, long k,
                                              const typename P::R (&x)[N],
                                              const typename P::R (&Pk)[N][N]) {
  using R = typename P::R;
  SElem<N, R> e;
  if (k == T - 1) {
    set_identity(e);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      e.E[i][i] = R(0);
      e.g[i] = x[i];
#pragma unroll
      for (int j = 0; j < N; ++j) e.L[i][j] = Pk[i][j];
    }
    return e;
  }
  R F[N][N], Q[N][N];
  load_mat<N, R>(tv.F + (k + 1) * N * N, F);
  load_mat<N, R>(tv.Q + (k + 1) * N * N, Q);
  e = smooth_element<N, P>(x, Pk, F, Q);
  if (tv.u) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      R s = R(0);
#pragma unroll
      for (int t = 0; t < N; ++t) s += e.E[i][t] * tv.u[(k + 1) * N + t];
      e.g[i] -= s;
    }
  }
  return e;
}

// The last block of a pass to finish resets the tile ticket and the finished
// count and advances the epoch, so the pass can be enqueued again without
// another preparation launch (its successor's tag differs from every tag this
// pass wrote).  Every block took its ticket and read the epoch before any
// block can be last.  The timeout flag (ctr[2]) is left for diagnosis.
KF_DEV void finish_grid(unsigned* __restrict__ ctr, unsigned* __restrict__ epoch, unsigned tag) {
  if (threadIdx.x == 0) {
    const unsigned done = atomicAdd(ctr + 1, 1u);
    if (done == gridDim.x - 1) {
      st_relaxed(ctr + 0, 0u);
      st_relaxed(ctr + 1, 0u);
      st_relaxed(epoch, tag);
    }
  }
}

// ===========================================================================
// Generic tile driver shared by the three scans.
//
// A pipeline P supplies, in scan order:
//   E                   element type; op(p, q) the scan-order combine
//   St                  anchored state (two arrays, v[N] and m[N][N]), the part
//                       of an anchored prefix/suffix the outputs need
//   fold(k0, tid)       the thread's aggregate over its L steps
//   apply(st, e)        st := st (x) e  (forward)   or  e (x) st  (reverse)
//   expand(st, e)       element form of an anchored state, for the look-back
//   anchor(e, st)       anchored state of an anchored element
//   initial(st)         the anchored state before tile 0 (scan order)
//   steps(k0, st)       apply the state step by step and write the outputs
// Tile 0 in scan order starts from initial(); it is the prior (m0, P0) for
// the time-invariant filter and the zero state elsewhere, which the anchored
// element inside tile 0 (step 1 for the filter, step T for the reverse
// scans) overwrites.
// ===========================================================================
template <int N, class R> struct St {
  R v[N];
  R m[N][N];
  static constexpr int SIZE = N + N * N;
};

template <int N, class R, class F> KF_DEV void each(St<N, R>& x, F f) {
  int k = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) f(x.v[i], k++);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) f(x.m[i][j], k++);
}

template <int N, class R> KF_DEV void st_zero(St<N, R>& s) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    s.v[i] = R(0);
#pragma unroll
    for (int j = 0; j < N; ++j) s.m[i][j] = R(0);
  }
}
template <int N, class R> KF_DEV void st_load(St<N, R>& s, const R* p) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    s.v[i] = p[i];
#pragma unroll
    for (int j = 0; j < N; ++j) s.m[i][j] = p[N + i * N + j];
  }
}
template <int N, class R> KF_DEV void st_store(R* p, const St<N, R>& s) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    p[i] = s.v[i];
#pragma unroll
    for (int j = 0; j < N; ++j) p[N + i * N + j] = s.m[i][j];
  }
}

// A pipeline may scan its wavefronts itself (TableScan<Pipe>::value): it
// then provides
//   scan_wave(tid, lane)  fold + wavefront inclusive scan; returns the lane's
//                         inclusive prefix (only the last lane's is used),
//                         keeping what lane_prefix needs in its own LDS
//   lane_prefix(tid)      the inclusive prefix of thread tid within its
//                         wavefront, as an element
// in place of the fold and of the generic wavefront scan below.
template <class Pipe, class = void> struct TableScan {
  static constexpr bool value = false;
};
template <class Pipe> struct TableScan<Pipe, std::void_t<decltype(Pipe::kTableScan)>> {
  static constexpr bool value = Pipe::kTableScan;
};

// A pipeline may also stage its loads and stores through LDS
// (StagesOut<Pipe>::value): its fold and its step walk then take the LDS of
// the per-thread wavefront prefixes as scratch (kStageBytes at most), each
// wavefront only the part that holds its own lanes' prefixes (so a
// wavefront that has finished its fold and scan never overwrites the
// scratch of one still folding), and the walk only after a workgroup
// barrier (the exclusive states have then been read).
template <class Pipe, class = void> struct StagesOut {
  static constexpr bool value = false;
};
template <class Pipe> struct StagesOut<Pipe, std::void_t<decltype(Pipe::kStageBytes)>> {
  static constexpr bool value = true;
};

template <class Pipe, int N, class R, int BLOCK, int L>
KF_DEV void scan_tile(Pipe& pp, const ScanArgs<R>& a) {
  using E = typename Pipe::E;
  constexpr bool TS = TableScan<Pipe>::value;
  constexpr int NW = BLOCK / WAVE;
  constexpr int PS = N + N * N;
  constexpr int ESW = E::SIZE * kWords<R>;  // tagged words per published element
  constexpr int PSW = PS * kWords<R>;       // tagged words per published anchored state
  __shared__ E s_wt[NW];               // inclusive totals of each wavefront
  __shared__ E s_x[TS ? 1 : BLOCK];    // inclusive prefix of each thread within its wavefront
  __shared__ R s_pre[PS];     // the tile's exclusive anchored state
  __shared__ E s_part[NW];    // look-back: wavefront partials of a window
  __shared__ int s_lp[NW];    // look-back: first lane of each wavefront with a published prefix
  __shared__ long s_tile, s_seq, s_t, s_base;
  __shared__ SeqInfo s_info;
  __shared__ unsigned s_tag;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
  if (tid == 0) {
    // The epoch word changes only when this pass's last workgroup finishes,
    // after every workgroup has started, so it is read before the ticket and
    // both are in flight together.
    const unsigned epoch = ld_relaxed(a.epoch);
    const long g = (long)atomicAdd(a.ctr, 1u);
    s_tile = g;
    s_tag = epoch + 1u;
    SeqInfo si;
    long sq, tt, bs;
    if (a.tile_seq) {
      sq = a.tile_seq[g];
      if (sq >= 0) {
        bs = (long)a.tile_start[sq];
        tt = g - bs;
        si.ntiles = (long)a.tile_start[sq + 1] - bs;
        si.T = (long)a.seq_len[sq];
        si.row0 = (long)a.seq_row[sq];
        si.model = a.cst_stride ? sq : 0;
      } else {
        bs = tt = 0;
        si = SeqInfo{0, 0, 0, 0};
      }
    } else {
      sq = g / a.ntiles;
      tt = g - sq * a.ntiles;
      bs = sq * a.ntiles;
      si = SeqInfo{a.T, a.ntiles, sq * a.T, 0};
    }
    s_seq = sq;
    s_t = tt;
    s_base = bs;
    s_info = si;
  }
  __syncthreads();
  const long gt = s_tile;
  const unsigned tag = s_tag;
  if (s_seq < 0) {  // a ragged batch's grid has spare blocks past the last tile
    finish_grid(a.ctr, a.epoch, tag);
    return;
  }
  // values read from LDS are the same in every lane; say so, so that the
  // pointers built from them stay scalar
  const long t = uniform(s_t);
  const long base = uniform(s_base);
  const SeqInfo si{uniform(s_info.T), uniform(s_info.ntiles), uniform(s_info.row0),
                   uniform(s_info.model)};
  pp.bind(si, t, tid);
  auto op = [&](const E& p, const E& q) { return pp.op(p, q); };

  // 1. thread fold
  if constexpr (TS) {
    E x = pp.scan_wave(tid, lane);
    if (lane == WAVE - 1) s_wt[wid] = x;
  } else {
    E x;
    if constexpr (StagesOut<Pipe>::value) x = pp.fold(reinterpret_cast<typename Pipe::R*>(s_x));
    else x = pp.fold();
    // 2. wavefront scan, results through LDS
    wave_inclusive_scan(x, lane, op);
    s_x[tid] = x;
    if (lane == WAVE - 1) s_wt[wid] = x;
  }
  __syncthreads();

  // 3. publish (wavefront 0; every lane holds the same values), look back
  //    (whole workgroup), publish the anchored inclusive prefix (wavefront 0).
  //    If a wavefront total is an anchor (decay_is_zero), the tile's anchored
  //    inclusive prefix follows from it and the later totals alone, so it is
  //    published at once, before the look-back; so is tile 0's, and so is
  //    the prefix of a tile whose aggregate is itself an anchor.  Otherwise
  //    the tile aggregate is published first and the prefix after the look-back.
  E tot;
  bool early = false;
  if (wid == 0) {
    int wa = -1;
#pragma unroll 1
    for (int w = NW - 1; w >= 0; --w)
      if (decay_is_zero(s_wt[w])) {
        wa = w;
        break;
      }
    if (t == 0 || wa >= 0) {
      St<N, R> st;
      if (wa >= 0) pp.anchor(s_wt[wa], st); else pp.initial(st);
#pragma unroll 1
      for (int w = wa + 1; w < NW; ++w) pp.apply(st, s_wt[w]);
      tag_publish<R>(a.pre + (base + t) * PSW, st, tag, lane);
      if (lane == 0) lb_publish_flag(a.flags + base + t, tag, LB_PREFIX);
      early = true;
    } else {
      tot = s_wt[0];
#pragma unroll 1
      for (int w = 1; w < NW; ++w) tot = op(tot, s_wt[w]);
      if (decay_is_zero(tot)) {
        St<N, R> st;
        pp.anchor(tot, st);
        tag_publish<R>(a.pre + (base + t) * PSW, st, tag, lane);
        if (lane == 0) lb_publish_flag(a.flags + base + t, tag, LB_PREFIX);
        early = true;
      } else {
        tag_publish<R>(a.agg + (base + t) * ESW, tot, tag, lane);
        if (lane == 0) lb_publish_flag(a.flags + base + t, tag, LB_AGG);
      }
    }
  }
  E ex;
  if (t > 0) {
    auto load_agg = [&](long idx, E& v) {
      tag_load<R>(v, a.agg + (base + idx) * ESW, tag, a.ctr + 2);
    };
    auto expand = [&](long idx, E& v) {
      St<N, R> sp;
      tag_load<R>(sp, a.pre + (base + idx) * PSW, tag, a.ctr + 2);
      pp.expand(sp, v);
    };
    auto try_expand = [&](long idx, E& v) {
      St<N, R> sp;
      const bool ok = tag_try_load<R>(sp, a.pre + (base + idx) * PSW, tag);
      pp.expand(sp, v);
      return ok;
    };
    // tiles per thread in a look-back window: one window of BLOCK*G tiles
    // reaches back over a whole sequence of up to 4*BLOCK tiles
    const long g = (si.ntiles + BLOCK - 1) / BLOCK;
    const int G = (int)(g < 1 ? 1 : (g > 4 ? 4 : g));
    ex = lookback<BLOCK, E>(a.flags + base, a.ctr + 2, tag, t, G, op, load_agg, expand,
                            try_expand, s_part, s_lp);
  }
  if (wid == 0 && t > 0) {
    St<N, R> st;
    pp.anchor(ex, st);
    if (lane == 0) st_store(s_pre, st);
    if (!early) {
      pp.apply(st, tot);
      tag_publish<R>(a.pre + (base + t) * PSW, st, tag, lane);
      if (lane == 0) lb_publish_flag(a.flags + base + t, tag, LB_PREFIX);
    }
  }
  __syncthreads();

  // 4. this thread's exclusive anchored state: the tile's, then the totals
  //    of the earlier wavefronts, then the earlier lanes of this wavefront,
  //    each starting over from the last anchor among them
  St<N, R> st;
  int ws = -1;
#pragma unroll 1
  for (int w = 0; w < wid; ++w)
    if (decay_is_zero(s_wt[w])) ws = w;
  if (ws >= 0) pp.anchor(s_wt[ws], st);
  else if (t > 0) st_load(st, s_pre);
  else pp.initial(st);
#pragma unroll 1
  for (int w = ws + 1; w < wid; ++w) pp.apply(st, s_wt[w]);
  if (lane > 0) {
    if constexpr (TS) {
      const E xp = pp.lane_prefix(tid - 1);
      if (decay_is_zero(xp)) pp.anchor(xp, st);
      else pp.apply(st, xp);
    } else {
      if (decay_is_zero(s_x[tid - 1])) pp.anchor(s_x[tid - 1], st);
      else pp.apply(st, s_x[tid - 1]);
    }
  }
  const bool have = (t > 0) || (tid > 0);
  if constexpr (StagesOut<Pipe>::value) {
    static_assert(TS || Pipe::kStageBytes <= sizeof(s_x), "staging exceeds the prefix buffer");
    pp.steps(st, have, reinterpret_cast<typename Pipe::R*>(s_x));
  } else {
    pp.steps(st, have);
  }
  finish_grid(a.ctr, a.epoch, tag);
}

// ---------------------------------------------------------------------------
// Forward filter (Algorithm 5): elements (eqs. pkf_init1..3), Lemma 1,
// anchored state (x_{k|k}, P_{k|k}) = (b, C) of a prefix that holds step 1.
// ---------------------------------------------------------------------------
template <int N, int M, class P, int L, bool TV = false> struct FilterPipe {
  using R = typename P::R;
  using E = FElem<N, R>;
  const ScanArgs<R>& a;
  const IO<R>& io;
  long T, k0;
  const R* __restrict__ cst;
  const R* __restrict__ y;
  R* __restrict__ mo;
  R* __restrict__ Po;
  const TvModel<R> tvm;
  KF_DEV FilterPipe(const ScanArgs<R>& a_, const IO<R>& io_, const TvModel<R>& tv_)
      : a(a_), io(io_), tvm(tv_) {}
  KF_DEV E element(long k, const R (&yk)[M]) const {
    if constexpr (TV) return filter_element_tv<N, M, P>(tvm, k, yk);
    else return filter_element<N, M, R>(cst, k, yk);
  }
  KF_DEV void bind(const SeqInfo& s, long t, int tid) {
    T = s.T;
    k0 = t * (long)(L * blockDim.x) + (long)tid * L;
    cst = io.cst + s.model * a.cst_stride;
    y = io.y + s.row0 * M;
    mo = io.m_out + s.row0 * N;
    Po = io.P_out + s.row0 * N * N;
  }
  KF_DEV E op(const E& p, const E& q) const { return fcombine<N, P>(p, q); }
  KF_DEV void load_y(long k, R (&yk)[M]) const {
#pragma unroll
    for (int c = 0; c < M; ++c) yk[c] = (k < T) ? y[k * M + c] : R(0);
  }
  // Steps are walked with the next step's measurement already in flight.
  KF_DEV E fold() const {
    E agg;
    set_identity(agg);
    R yn[M];
    load_y(k0, yn);
#pragma unroll 1
    for (int i = 0; i < L; ++i) {
      const long k = k0 + i;
      if (k >= T) break;
      R yk[M];
      copy_vec<M, R>(yn, yk);
      load_y(k + 1, yn);
      E el = element(k, yk);
      agg = (i == 0) ? el : fcombine<N, P>(agg, el);
    }
    return agg;
  }
  KF_DEV void apply(St<N, R>& st, const E& e) const { fapply<N, P>(st.v, st.m, e); }
  KF_DEV void initial(St<N, R>& st) const { st_zero(st); }
  KF_DEV void anchor(const E& e, St<N, R>& st) const {
    copy_vec<N, R>(e.b, st.v);
    copy_mat<N, N, R>(e.C, st.m);
  }
  KF_DEV void expand(const St<N, R>& st, E& v) const {
    set_identity(v);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      v.A[i][i] = R(0);
      v.b[i] = st.v[i];
#pragma unroll
      for (int j = 0; j < N; ++j) v.C[i][j] = st.m[i][j];
    }
  }
  KF_DEV void steps(St<N, R>& st, bool) const {
    R yn[M];
    load_y(k0, yn);
#pragma unroll 1
    for (int i = 0; i < L; ++i) {
      const long k = k0 + i;
      if (k >= T) break;
      R yk[M];
      copy_vec<M, R>(yn, yk);
      load_y(k + 1, yn);
      fapply<N, P>(st.v, st.m, element(k, yk));
      st_store_out(k, st);
    }
  }
  KF_DEV void st_store_out(long k, const St<N, R>& st) const {
#pragma unroll
    for (int r = 0; r < N; ++r) {
      st_out(&mo[k * N + r], st.v[r]);
#pragma unroll
      for (int c = 0; c < N; ++c) st_out(&Po[k * N * N + r * N + c], st.m[r][c]);
    }
  }
};

#define KFS_IO_PARAMS(R)                                                                  \
  const R* __restrict__ cst, const R* __restrict__ y, const R* __restrict__ m_in,        \
      const R* __restrict__ P_in, R* __restrict__ m_out, R* __restrict__ P_out
#define KFS_IO_MAKE(R) const IO<R> io{cst, y, m_in, P_in, m_out, P_out}

template <int N, int M, class P, int BLOCK, int L, bool TV = false>
__global__ __launch_bounds__(BLOCK) void k_filter(ScanArgs<typename P::R> a,
                                                  TvModel<typename P::R> tv,
                                                  KFS_IO_PARAMS(typename P::R)) {
  KFS_IO_MAKE(typename P::R);
  FilterPipe<N, M, P, L, TV> pp(a, io, tv);
  scan_tile<FilterPipe<N, M, P, L, TV>, N, typename P::R, BLOCK, L>(pp, a);
}

// ---------------------------------------------------------------------------
// Time-invariant forward filter (Algorithm 5 for a model with constant F, Q,
// H, R).  The prior is taken as the anchored state before step 1, so every
// step carries the generic element of eq. pkf_init1 (the element of eq.
// pkf_init2 equals (0, m0, P0) (x) that generic element).  By Lemma 1 the
// matrix part of an aggregate of L consecutive generic elements is the same
// for every thread (SL) and its vector part is linear in the measurements,
// so a thread's fold is  b = sum_i PHI[i] y_i, eta = sum_i PSI[i] y_i.  Steps
// past T are padded with y = 0; the filter is causal, so the outputs at
// valid steps are unaffected and the padded ones are not written.  The
// per-step apply is the Kalman predict/update (kf_step).
//
// The same holds one level up.  Every thread aggregate covers L generic
// elements, so the matrix part of any run of c consecutive thread
// aggregates is the same in every wavefront and tile: S_{cL} (A, C, J of c*L
// generic elements), and the vector part of a Lemma 1 combine of a run of a
// aggregates with a later run of c is linear in the operands' vector parts,
//   b = P1 b_x + P2 eta_y + b_y,   eta = P3 eta_y - P4 b_x + eta_x,
// with coefficients P1..P4 that depend on (a, c) only (mpart_combine_lanes).
// The wavefront scan (Hillis-Steele, offsets 2^d) only ever combines a run of
// a = min(l - 2^d + 1, 2^d) aggregates with one of 2^d, so each workgroup
// first builds S_{cL} for c = 1..64 and the coefficients of those 63 pairs
// in LDS, level by level, 16 lanes per combine (in precision P::S, from the
// FP64-derived S_L of the model constants); the threads then fold and scan
// only the vector parts (b, eta), with no factorisation per lane.  A lane's
// prefix is rebuilt as an element (S_{cL} with its vector part) where the
// look-back and the exclusive states need one.
template <int N, int M, class P, int L, int BLOCK> struct FilterTiPipe {
  using R = typename P::R;
  using S = typename P::S;
  using E = FElem<N, R>;
  using LY = CL<N, M, L>;
  static constexpr bool kTableScan = N * N <= 16;
  static constexpr int NGRP = BLOCK / 16;  // 16-lane groups, one combine each
  // Lanes read different entries of each table at once, so every entry is
  // padded: consecutive entries then start in different LDS banks instead
  // of all in the same one.  The coefficient rows are read as 16-byte
  // vectors, so those entries are padded by 16 bytes and kept aligned.
  struct Agg {
    MPart<N, S> m;
    S pad;
  };
  struct alignas(16) Coef {
    S c[4][N][N];
    S pad[16 / sizeof(S)];
  };
  struct Vec {
    R v[2 * N];
    R pad;
  };
  struct Tables {
    Agg agg[WAVE];                    // agg[c - 1].m = S_{cL}
    Coef coef[WAVE - 1];              // P1..P4 of (a, 2^d) at index 2^d - 1 + a - 1
    S work[NGRP][4][N][N];            // combine scratch of each group
    Vec v[BLOCK];                     // (b, eta) of each lane's inclusive prefix
  };
  // Output staging of the step walk: each wavefront's rows of SB consecutive
  // steps per lane (RW scalars each, lane l's rows padded by l scalars so
  // that the lanes' rows start in different banks).  The walk starts after
  // the last read of the tables, so the two share their LDS.
  static constexpr int RW = N + N * N;
  static constexpr int SB = (sizeof(R) == 4 ? 4 : 2) < L ? (sizeof(R) == 4 ? 4 : 2) : L;
  static constexpr int STG = WAVE * SB * RW + WAVE;
  union Shared {
    Tables t;
    R stg[BLOCK / WAVE][STG];
  };
  KF_DEV static Shared& shared() {
    __shared__ Shared sh;
    return sh;
  }
  KF_DEV static Tables& tables() { return shared().t; }
  const ScanArgs<R>& a;
  const IO<R>& io;
  long T, k0;
  const R* __restrict__ cst;
  R* __restrict__ mo;
  R* __restrict__ Po;
  R yv[L][M];
  KF_DEV FilterTiPipe(const ScanArgs<R>& a_, const IO<R>& io_) : a(a_), io(io_) {}
  // Vector loads complete in order, so the first table entry S_L, which
  // the table build waits for, is requested before the measurements, which
  // are not needed until the fold.  The measurement loads are unconditional
  // (a padded step reads the sequence's last row, and its value is then
  // replaced by zero): a load under a per-step branch would have to complete
  // before the branches merge, one round trip after another.
  KF_DEV void bind(const SeqInfo& s, long t, int tid) {
    T = s.T;
    k0 = t * (long)(L * blockDim.x) + (long)tid * L;
    cst = io.cst + s.model * a.cst_stride;
    const R* __restrict__ y = io.y + s.row0 * M;
    mo = io.m_out + s.row0 * N;
    Po = io.P_out + s.row0 * N * N;
    S sl[3] = {S(0), S(0), S(0)};
    if (tid < N * N)
#pragma unroll
      for (int q = 0; q < 3; ++q) sl[q] = S(cst[LY::SL + q * N * N + tid]);
    // a workgroup has a tile only in a sequence with T >= 1
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const bool in = k0 + i < T;
      const long k = in ? k0 + i : T - 1;
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const R v = y[k * M + c];
        yv[i][c] = in ? v : R(0);
      }
    }
    if (tid < N * N) {
      Tables& tb = tables();
      const int r = tid / N, j = tid % N;
      tb.agg[0].m.A[r][j] = sl[0];
      tb.agg[0].m.C[r][j] = sl[1];
      tb.agg[0].m.J[r][j] = sl[2];
    }
  }
  KF_DEV E op(const E& p, const E& q) const { return fcombine<N, P>(p, q); }
  // S_{cL} as an element with vector part v = (b, eta)
  KF_DEV static E with_vector(const MPart<N, S>& m, const R* v) {
    E e;
#pragma unroll
    for (int r = 0; r < N; ++r) {
      e.b[r] = v[r];
      e.e[r] = v[N + r];
#pragma unroll
      for (int j = 0; j < N; ++j) {
        e.A[r][j] = R(m.A[r][j]);
        e.C[r][j] = R(m.C[r][j]);
        e.J[r][j] = R(m.J[r][j]);
      }
    }
    return e;
  }
  KF_DEV E scan_wave(int tid, int lane) const {
    Tables& tb = tables();
    // S_L, written by bind
    __syncthreads();
    // level d: S_{(a + h)L} = S_{aL} (x) S_{hL} and its coefficients, h = 2^d,
    // a = 1..h; the inputs come from earlier levels
    const int grp = tid >> 4, gl = tid & 15;
#pragma unroll 1
    for (int h = 1; h < WAVE; h <<= 1) {
#pragma unroll 1
      for (int a0 = 0; a0 < h; a0 += NGRP) {
        const int a = a0 + grp + 1;
        const bool act = a <= h;
        const int ai = act ? a : 1;
        mpart_combine_lanes<N, S>(tb.agg[ai - 1].m, tb.agg[h - 1].m, tb.agg[act ? ai + h - 1 : 0].m,
                                  tb.coef[h - 1 + ai - 1].c, tb.work[grp], act ? gl : 16);
      }
      __syncthreads();
    }
    // fold and scan the vector parts
    R b[N], e[N];
    fold_vec(b, e);
#pragma unroll 1
    for (int h = 1; h < WAVE; h <<= 1) {
      R ub[N], ue[N];
#pragma unroll
      for (int r = 0; r < N; ++r) {
        ub[r] = __shfl_up(b[r], h, WAVE);
        ue[r] = __shfl_up(e[r], h, WAVE);
      }
      if (lane >= h) {
        const int a = (lane - h + 1 < h) ? lane - h + 1 : h;
        const S (&Pc)[4][N][N] = tb.coef[h - 1 + a - 1].c;
        R nb[N], ne[N];
#pragma unroll
        for (int r = 0; r < N; ++r) {
          S sb = S(b[r]), se = S(ue[r]);
#pragma unroll
          for (int t = 0; t < N; ++t) {
            sb += Pc[0][r][t] * S(ub[t]) + Pc[1][r][t] * S(e[t]);
            se += Pc[2][r][t] * S(e[t]) - Pc[3][r][t] * S(ub[t]);
          }
          nb[r] = R(sb);
          ne[r] = R(se);
        }
        copy_vec<N, R>(nb, b);
        copy_vec<N, R>(ne, e);
      }
    }
#pragma unroll
    for (int r = 0; r < N; ++r) {
      tb.v[tid].v[r] = b[r];
      tb.v[tid].v[N + r] = e[r];
    }
    return with_vector(tb.agg[lane].m, tb.v[tid].v);
  }
  KF_DEV E lane_prefix(int t) const {
    Tables& tb = tables();
    return with_vector(tb.agg[t & (WAVE - 1)].m, tb.v[t].v);
  }
  // vector part of the thread's aggregate of L generic elements
  KF_DEV void fold_vec(R (&b)[N], R (&e)[N]) const {
    const R* __restrict__ c = cst;
#pragma unroll
    for (int r = 0; r < N; ++r) {
      R sb = R(0), se = R(0);
#pragma unroll
      for (int i = 0; i < L; ++i)
#pragma unroll
        for (int q = 0; q < M; ++q) {
          sb += c[LY::PHI + i * N * M + r * M + q] * yv[i][q];
          se += c[LY::PSI + i * N * M + r * M + q] * yv[i][q];
        }
      b[r] = sb;
      e[r] = se;
    }
  }
  KF_DEV E fold() const {
    const R* __restrict__ c = cst;
    E e;
#pragma unroll
    for (int r = 0; r < N; ++r) {
      R b = R(0), h = R(0);
#pragma unroll
      for (int i = 0; i < L; ++i)
#pragma unroll
        for (int q = 0; q < M; ++q) {
          b += c[LY::PHI + i * N * M + r * M + q] * yv[i][q];
          h += c[LY::PSI + i * N * M + r * M + q] * yv[i][q];
        }
      e.b[r] = b;
      e.e[r] = h;
#pragma unroll
      for (int j = 0; j < N; ++j) {
        e.A[r][j] = c[LY::SL + r * N + j];
        e.C[r][j] = c[LY::SL + N * N + r * N + j];
        e.J[r][j] = c[LY::SL + 2 * N * N + r * N + j];
      }
    }
    return e;
  }
  KF_DEV void apply(St<N, R>& st, const E& e) const { fapply<N, P>(st.v, st.m, e); }
  KF_DEV void initial(St<N, R>& st) const {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      st.v[i] = cst[LY::m0 + i];
#pragma unroll
      for (int j = 0; j < N; ++j) st.m[i][j] = cst[LY::P0 + i * N + j];
    }
  }
  KF_DEV void anchor(const E& e, St<N, R>& st) const {
    copy_vec<N, R>(e.b, st.v);
    copy_mat<N, N, R>(e.C, st.m);
  }
  KF_DEV void expand(const St<N, R>& st, E& v) const {
    set_identity(v);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      v.A[i][i] = R(0);
      v.b[i] = st.v[i];
#pragma unroll
      for (int j = 0; j < N; ++j) v.C[i][j] = st.m[i][j];
    }
  }
  // The walk: L Kalman steps per thread, in blocks of SB steps.  The
  // outputs of a block are staged in LDS and then leave in whole runs: the
  // rows of lane g's block are contiguous in memory (SB rows), and the
  // wavefront stores them with consecutive lanes on consecutive chunks of up
  // to 16 bytes, so each store instruction writes few, whole lines instead
  // of one piece of 64 different lines.
  KF_DEV void steps(St<N, R>& st, bool) const {
    R F[N][N], Q[N][N], H[M][N], Rm[M][M];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) {
        F[i][j] = cst[LY::F + i * N + j];
        Q[i][j] = cst[LY::Q + i * N + j];
      }
#pragma unroll
    for (int i = 0; i < M; ++i) {
#pragma unroll
      for (int j = 0; j < N; ++j) H[i][j] = cst[LY::H + i * N + j];
#pragma unroll
      for (int j = 0; j < M; ++j) Rm[i][j] = cst[LY::Rm + i * M + j];
    }
    __syncthreads();  // every lane is done with the tables
    const int lane = threadIdx.x & (WAVE - 1);
    R* stg = shared().stg[threadIdx.x / WAVE];
#pragma unroll
    for (int s0 = 0; s0 < L; s0 += SB) {
#pragma unroll
      for (int i = 0; i < SB; ++i) {
        if (k0 + s0 + i < T) kf_step<N, M, P>(st.v, st.m, F, Q, H, Rm, yv[s0 + i]);
        R* row = stg + (lane * SB + i) * RW + lane;
#pragma unroll
        for (int r = 0; r < N; ++r) {
          row[r] = st.v[r];
#pragma unroll
          for (int c = 0; c < N; ++c) row[N + r * N + c] = st.m[r][c];
        }
      }
      wave_lds_sync();
      store_block<N * N, N>(stg, s0, Po);
      store_block<N, 0>(stg, s0, mo);
      wave_lds_sync();
    }
  }
  // chunk of a run of W-scalar rows: up to 16 bytes, dividing the row
  template <int W> static constexpr int chunk() {
    return (W * (int)sizeof(R)) % 16 == 0 ? 16 / (int)sizeof(R)
           : (W * (int)sizeof(R)) % 8 == 0 ? (8 / (int)sizeof(R) > 0 ? 8 / (int)sizeof(R) : 1)
                                           : 1;
  }
  // Store the staged block (steps s0 .. s0+SB-1 of every lane of the
  // wavefront) of the output with W scalars per row, found at scalar OFF of
  // each staged row.
  template <int W, int OFF> KF_DEV void store_block(const R* stg, int s0, R* out) const {
    constexpr int CH = chunk<W>();
    constexpr int PER = SB * W / CH;  // chunks per lane's run
    const int lane = threadIdx.x & (WAVE - 1);
    const long wk0 = k0 - (long)lane * L;  // first row of the wavefront
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int c = j * WAVE + lane;
      const int g = c / PER, o = (c % PER) * CH;
      const int row = o / W, e = o % W;
      const long k = wk0 + (long)g * L + s0 + row;
      if (k < T) {
        const R* q = stg + (g * SB + row) * RW + g + OFF + e;
        R v[CH];
#pragma unroll
        for (int t = 0; t < CH; ++t) v[t] = q[t];
        __builtin_memcpy(out + k * W + e, v, sizeof(v));
      }
    }
  }
};

template <int N, int M, class P, int BLOCK, int L>
__global__ __launch_bounds__(BLOCK) void k_filter_ti(ScanArgs<typename P::R> a,
                                                     KFS_IO_PARAMS(typename P::R)) {
  KFS_IO_MAKE(typename P::R);
  FilterTiPipe<N, M, P, L, BLOCK> pp(a, io);
  scan_tile<FilterTiPipe<N, M, P, L, BLOCK>, N, typename P::R, BLOCK, L>(pp, a);
}

// ---------------------------------------------------------------------------
// RTS smoother reverse scan (Algorithm 6).  Scan order is descending time:
// tile t (scan order) covers time tile ntiles-1-t, thread tid covers time
// chunk BLOCK-1-tid of it and walks its steps from last to first.  Anchored
// state (x_{k|T}, P_{k|T}) = (g, L) of a suffix that holds step T.
// ---------------------------------------------------------------------------
template <int N, class R> KF_DEV void load_state(const R* __restrict__ m, const R* __restrict__ Pm,
                                                  long k, R (&x)[N], R (&P)[N][N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    x[i] = m[k * N + i];
#pragma unroll
    for (int j = 0; j < N; ++j) P[i][j] = Pm[k * N * N + i * N + j];
  }
}

// Smoothing element of row k from the filter moments (x, Pk) of that row:
// eq. prts_init2 at the last row, eq. prts_init1 elsewhere.
template <int N, int M, class P>
KF_DEV SElem<N, typename P::R> rts_element(const typename P::R* __restrict__ cst, long T, long k,
                                           const typename P::R (&x)[N],
                                           const typename P::R (&Pk)[N][N]) {
  using R = typename P::R;
  using LY = CL<N, M>;
  SElem<N, R> e;
  if (k == T - 1) {
    set_identity(e);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      e.E[i][i] = R(0);
      e.g[i] = x[i];
#pragma unroll
      for (int j = 0; j < N; ++j) e.L[i][j] = Pk[i][j];
    }
  } else {
    R Fm[N][N], Qm[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) {
        Fm[i][j] = cst[LY::F + i * N + j];
        Qm[i][j] = cst[LY::Q + i * N + j];
      }
    e = smooth_element<N, P>(x, Pk, Fm, Qm);
  }
  return e;
}

// Element at row k of the two-filter backward scan over (a_2, ..., a_T, e):
// a_{k+2} built from y at row k+1, the identity at the last row.
template <int N, int M, class R>
KF_DEV FElem<N, R> tf_element(const R* __restrict__ cst, long T, long k, const R (&yk)[M]) {
  FElem<N, R> e;
  if (k == T - 1) set_identity(e);
  else e = filter_element<N, M, R>(cst, k + 1, yk);
  return e;
}

template <int N, int M, class P, int L, int B, bool TV = false> struct RtsPipe {
  using R = typename P::R;
  using E = SElem<N, R>;
  using LY = CL<N, M>;
  const ScanArgs<R>& a;
  const IO<R>& io;
  long T, k0;
  const R* __restrict__ cst;
  const R* __restrict__ mf;
  const R* __restrict__ Pf;
  R* __restrict__ mo;
  R* __restrict__ Po;
  const TvModel<R> tvm;
  KF_DEV RtsPipe(const ScanArgs<R>& a_, const IO<R>& io_, const TvModel<R>& tv_)
      : a(a_), io(io_), tvm(tv_) {}
  KF_DEV void bind(const SeqInfo& s, long t, int tid) {
    T = s.T;
    const long tt = s.ntiles - 1 - t;
    k0 = tt * (long)(L * blockDim.x) + (long)(blockDim.x - 1 - tid) * L;
    cst = io.cst + s.model * a.cst_stride;
    mf = io.m_in + s.row0 * N;
    Pf = io.P_in + s.row0 * N * N;
    mo = io.m_out + s.row0 * N;
    Po = io.P_out + s.row0 * N * N;
  }
  // p precedes q in scan order, so p is the later one in time
  KF_DEV E op(const E& p, const E& q) const { return scombine<N, P>(q, p); }
  KF_DEV void load(long k, R (&x)[N], R (&Pk)[N][N]) const {
    if (k >= 0 && k < T) load_state<N, R>(mf, Pf, k, x, Pk);
  }
  KF_DEV E element(long k, const R (&x)[N], const R (&Pk)[N][N]) const {
    if constexpr (TV) return rts_element_tv<N, P>(tvm, T, k, x, Pk);
    else return rts_element<N, M, P>(cst, T, k, x, Pk);
  }
  // Steps are walked last to first in groups of PG consecutive rows whose
  // covariances fill one 128-byte line (two rows at nx = 4 in FP32), with the
  // next (earlier) group already in flight.  In FP32 a thread's L filtered
  // means are read once into an LDS column of its own, serve both walks, and
  // are overwritten in place by the smoothed means.
  static constexpr int PG = (N * N * (int)sizeof(R) <= 64 && L % 2 == 0) ? 2 : 1;
  static constexpr int NG = L / PG;
  static constexpr bool MLDS = (sizeof(R) == 4);
  R* ms;  // this thread's column: row i, component c at ms[(i * N + c) * B]
  KF_DEV void mean_rows(long kb, int ib, R (&x)[PG][N]) const {
    if (MLDS) {
#pragma unroll
      for (int i = 0; i < PG; ++i)
#pragma unroll
        for (int r = 0; r < N; ++r) x[i][r] = ms[((ib + i) * N + r) * B];
    }
  }
  // Filtered covariances are read a group at a time by the whole
  // wavefront: each lane's PG rows are contiguous in memory, so the
  // wavefront loads them with consecutive lanes on consecutive 16-byte
  // chunks (whole lines per load instruction) into registers, one group
  // ahead, and passes them through its LDS staging to the lanes that own
  // them.  In FP32 the wavefront's filtered means (64 * L consecutive rows)
  // are read the same way into the threads' LDS columns.
  static constexpr int CHP = (N * N * (int)sizeof(R)) % 16 == 0 ? 16 / (int)sizeof(R)
                             : ((N * N * (int)sizeof(R)) % 8 == 0 && sizeof(R) == 4) ? 2
                                                                                   : 1;
  static constexpr int PERP = PG * N * N / CHP;  // chunks of a lane's group, one per load pass
  // A load pass covers LPP lanes' groups, PERP lanes each (the last lanes
  // idle when PERP does not divide 64): in pass j, lane sub * PERP + q takes
  // chunk q of lane l = j * LPP + sub, whose rows start LPP * L rows lower
  // for every further pass -- one base address per lane and a fixed stride
  // between passes.
  static constexpr int LPP = WAVE / PERP;
  static constexpr int NP = (WAVE + LPP - 1) / LPP;  // load passes per group
  KF_DEV void fetch_group(int g, R (&buf)[NP][CHP]) const {
    const int lane = threadIdx.x & (WAVE - 1);
    const int sub = lane / PERP, o = (lane % PERP) * CHP;
    const long kb = lane_k0(sub) + g * PG + o / NN;  // pass 0
    const R* src = Pf + kb * NN + o % NN;
    constexpr long STEP = (long)LPP * L * NN;  // scalars between passes
    // all rows below T unless this is the sequence's last tile
    const bool all = uniform(lane_k0(0) + L - 1) < T;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const bool act = sub < LPP && j * LPP + sub < WAVE;
      if (act && (all || kb - (long)j * LPP * L < T)) {
        __builtin_memcpy(buf[j], src - j * STEP, sizeof(buf[j]));
      } else {
#pragma unroll
        for (int t = 0; t < CHP; ++t) buf[j][t] = R(0);
      }
    }
  }
  // put the fetched chunks in the staging rows, then read this lane's rows
  KF_DEV void unstage_group(R* stg, const R (&buf)[NP][CHP], R (&Pk)[PG][N][N]) const {
    const int lane = threadIdx.x & (WAVE - 1);
    const int sub = lane / PERP, o = (lane % PERP) * CHP;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const int l = j * LPP + sub;
      if (sub < LPP && l < WAVE) {
        R* q = stg + (l * PG + o / NN) * NN + l + o % NN;
#pragma unroll
        for (int t = 0; t < CHP; ++t) q[t] = buf[j][t];
      }
    }
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < PG; ++i)
#pragma unroll
      for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c < N; ++c) Pk[i][r][c] = stg[(lane * PG + i) * NN + lane + r * N + c];
    wave_lds_sync();
  }
  KF_DEV void load_means() {
    __shared__ R s_mean[MLDS ? L * N * B : 1];
    ms = s_mean + threadIdx.x;
    constexpr int CH = chunk<N>();
    constexpr int PER = N / CH;
    constexpr int NJ = L * PER;
    const int lane = threadIdx.x & (WAVE - 1);
    const long base = lane_k0(WAVE - 1);
    R* col0 = ms - lane;
    // Every load is issued before the first LDS write: a value stored as
    // soon as it is loaded would be waited for before the next load went
    // out.  Chunk j of lane `lane` is chunk c = j * WAVE + lane of the
    // wavefront's rows base .. base + WAVE * L - 1, at offset c * CH from
    // row base.  Rows past T are read from row T - 1 (a sequence has at
    // least one step) and replaced by zeros.
    R v[NJ][CH];
    if (uniform(base + (long)WAVE * L - 1) < T) {
      const R* p = mf + base * N + lane * CH;
#pragma unroll
      for (int j = 0; j < NJ; ++j) __builtin_memcpy(v[j], p + j * WAVE * CH, sizeof(v[j]));
    } else {
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int c = j * WAVE + lane;
        const int e = (c % PER) * CH;
        const long k = base + c / PER;
        const bool in = k < T;
        __builtin_memcpy(v[j], mf + (in ? k : T - 1) * N + e, sizeof(v[j]));
#pragma unroll
        for (int t = 0; t < CH; ++t) v[j][t] = in ? v[j][t] : R(0);
      }
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int c = j * WAVE + lane;
      const int rr = c / PER, e = (c % PER) * CH;
      const int l = WAVE - 1 - rr / L, i = rr % L;
#pragma unroll
      for (int t = 0; t < CH; ++t) col0[(i * N + e + t) * B + l] = v[j][t];
    }
    wave_lds_sync();
  }
  KF_DEV void load_x(int g, R (&x)[PG][N]) const {
#pragma unroll
    for (int i = 0; i < PG; ++i) {
      const long k = k0 + g * PG + i;
#pragma unroll
      for (int r = 0; r < N; ++r) x[i][r] = (k < T) ? mf[k * N + r] : R(0);
    }
  }
  KF_DEV E fold(R* stage) {
    E agg;
    set_identity(agg);
    R* stg = stage + (threadIdx.x / WAVE) * WSTR;
    R buf[NP][CHP], xn[PG][N];
    fetch_group(NG - 1, buf);
    if (MLDS) load_means();
    else load_x(NG - 1, xn);
#pragma unroll 1
    for (int g = NG - 1; g >= 0; --g) {
      R x[PG][N], Pk[PG][N][N];
      unstage_group(stg, buf, Pk);
      if (MLDS) {
        if (g > 0) fetch_group(g - 1, buf);
        mean_rows(k0 + g * PG, g * PG, x);
      } else {
#pragma unroll
        for (int i = 0; i < PG; ++i) copy_vec<N, R>(xn[i], x[i]);
        if (g > 0) {
          fetch_group(g - 1, buf);
          load_x(g - 1, xn);
        }
      }
#pragma unroll
      for (int i = PG - 1; i >= 0; --i) {
        const long k = k0 + g * PG + i;
        if (k < T) agg = scombine<N, P>(element(k, x[i], Pk[i]), agg);
      }
    }
    return agg;
  }
  KF_DEV void apply(St<N, R>& st, const E& e) const { sapply<N, P>(e, st.v, st.m); }
  KF_DEV void initial(St<N, R>& st) const { st_zero(st); }
  KF_DEV void anchor(const E& e, St<N, R>& st) const {
    copy_vec<N, R>(e.g, st.v);
    copy_mat<N, N, R>(e.L, st.m);
  }
  KF_DEV void expand(const St<N, R>& st, E& v) const {
    set_identity(v);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      v.E[i][i] = R(0);
      v.g[i] = st.v[i];
#pragma unroll
      for (int j = 0; j < N; ++j) v.L[i][j] = st.m[i][j];
    }
  }
  // Same grouping as fold().  A group's smoothed covariances (PG rows per
  // lane, contiguous in memory) are staged in LDS and stored by the whole
  // wavefront with consecutive lanes on consecutive 16-byte chunks, so each
  // store instruction writes whole lines; in FP32 the smoothed means collect
  // in the thread's LDS column and leave at the end as one contiguous run per
  // wavefront (its 64 threads own 64 * L consecutive rows).
  static constexpr int NN = N * N;
  static constexpr int STG = WAVE * PG * NN + WAVE;  // per wavefront, lane rows padded by lane
  // a wavefront's staging starts where its lanes' wavefront prefixes do
  static constexpr int WSTR = WAVE * (int)sizeof(E) / (int)sizeof(R);
  static_assert(STG <= WSTR, "staging of a wavefront exceeds its prefix slots");
  static constexpr size_t kStageBytes = (size_t)(B / WAVE) * WSTR * sizeof(R);
  template <int W> static constexpr int chunk() {
    return (W * (int)sizeof(R)) % 16 == 0 ? 16 / (int)sizeof(R)
           : ((W * (int)sizeof(R)) % 8 == 0 && sizeof(R) == 4) ? 2
                                                               : 1;
  }
  KF_DEV void steps(St<N, R>& st, bool, R* stage) const {
    __syncthreads();  // every lane has read its prefix from the staging space
    const int lane = threadIdx.x & (WAVE - 1);
    R* stg = stage + (threadIdx.x / WAVE) * WSTR;
    R buf[NP][CHP], xn[PG][N];
    fetch_group(NG - 1, buf);
    if (!MLDS) load_x(NG - 1, xn);
#pragma unroll 1
    for (int g = NG - 1; g >= 0; --g) {
      R x[PG][N], Pk[PG][N][N];
      unstage_group(stg, buf, Pk);
      if (MLDS) {
        if (g > 0) fetch_group(g - 1, buf);
        mean_rows(k0 + g * PG, g * PG, x);
      } else {
#pragma unroll
        for (int i = 0; i < PG; ++i) copy_vec<N, R>(xn[i], x[i]);
        if (g > 0) {
          fetch_group(g - 1, buf);
          load_x(g - 1, xn);
        }
      }
#pragma unroll
      for (int i = PG - 1; i >= 0; --i) {
        const long k = k0 + g * PG + i;
        if (k < T) sapply<N, P>(element(k, x[i], Pk[i]), st.v, st.m);
        R* row = stg + (lane * PG + i) * NN + lane;
#pragma unroll
        for (int r = 0; r < N; ++r)
#pragma unroll
          for (int c = 0; c < N; ++c) row[r * N + c] = st.m[r][c];
        if (MLDS) {
#pragma unroll
          for (int r = 0; r < N; ++r) ms[((g * PG + i) * N + r) * B] = st.v[r];
        } else if (k < T) {
#pragma unroll
          for (int r = 0; r < N; ++r) st_out(&mo[k * N + r], st.v[r]);
        }
      }
      wave_lds_sync();
      store_cov_group(stg, g);
      wave_lds_sync();
    }
    if (MLDS) store_means();
  }
  // Lane l of this wavefront holds rows k0(l) .. k0(l) + L - 1 with
  // k0(l) = k0 + (lane - l) * L (the walk's threads run in descending
  // time), so row k0(l) + j is row (63 - l) * L + j of the wavefront's run.
  KF_DEV long lane_k0(int l) const {
    const int lane = threadIdx.x & (WAVE - 1);
    return k0 + (long)(lane - l) * L;
  }
  KF_DEV void store_cov_group(const R* stg, int g) const {
    constexpr int CH = chunk<NN>();
    constexpr int PER = PG * NN / CH;
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int c = j * WAVE + lane;
      const int l = c / PER, o = (c % PER) * CH;
      const int row = o / NN, e = o % NN;
      const long k = lane_k0(l) + g * PG + row;
      if (k < T) {
        const R* q = stg + (l * PG + row) * NN + l + e;
        R v[CH];
#pragma unroll
        for (int t = 0; t < CH; ++t) v[t] = q[t];
        __builtin_memcpy(Po + k * NN + e, v, sizeof(v));
      }
    }
  }
  // FP32 smoothed means, from the LDS columns of the wavefront's threads:
  // the wavefront's rows are contiguous, row r of the run belongs to the
  // thread whose k0 is the largest not above it.
  KF_DEV void store_means() const {
    constexpr int CH = chunk<N>();
    constexpr int PER = N / CH;
    const int lane = threadIdx.x & (WAVE - 1);
    const long base = lane_k0(WAVE - 1);  // lowest row of the wavefront
    const R* col0 = ms - lane;            // column of lane 0 of this wavefront
#pragma unroll
    for (int j = 0; j < L * PER; ++j) {
      const int c = j * WAVE + lane;
      const int rr = c / PER, e = (c % PER) * CH;
      const long k = base + rr;
      const int l = WAVE - 1 - rr / L, i = rr % L;
      if (k < T) {
        R v[CH];
#pragma unroll
        for (int t = 0; t < CH; ++t) v[t] = col0[((i * N + e + t) * B) + l];
        __builtin_memcpy(mo + k * N + e, v, sizeof(v));
      }
    }
  }
};

// Two workgroups per CU in FP32 (the grid of the long sequences is two
// tiles per CU); the wider precisions keep the register budget of one.
template <class P> constexpr int rts_min_blocks() { return sizeof(typename P::S) == 4 ? 2 : 1; }

template <int N, int M, class P, int BLOCK, int L, bool TV = false>
__global__ __launch_bounds__(BLOCK, rts_min_blocks<P>()) void k_rts(ScanArgs<typename P::R> a, TvModel<typename P::R> tv,
                                               KFS_IO_PARAMS(typename P::R)) {
  KFS_IO_MAKE(typename P::R);
  RtsPipe<N, M, P, L, BLOCK, TV> pp(a, io, tv);
  scan_tile<RtsPipe<N, M, P, L, BLOCK, TV>, N, typename P::R, BLOCK, L>(pp, a);
}

// ---------------------------------------------------------------------------
// Two-filter smoother backward pass (Algorithm 7): reverse scan over
// (a_2, ..., a_T, e) with the filtering operator; position k (0-based row)
// holds a_{k+2} for k < T-1 and the identity e at k = T-1, so the suffix at
// row k is a_{k+2} (x) ... (x) a_T (x) e, whose (eta, J) is eta_{k+1|k+2:T},
// J_{k+1|k+2:T}.  The anchored state is that (eta, J); the combination with
// the filter result (m_in, P_in) is fused into the step phase.
// ---------------------------------------------------------------------------
template <int N, int M, class P, int L, bool TI, bool TV = false> struct TwoFilterPipe {
  using R = typename P::R;
  using E = FElem<N, R>;
  const ScanArgs<R>& a;
  const IO<R>& io;
  long T, k0;
  const R* __restrict__ cst;
  const R* __restrict__ y;
  const R* __restrict__ mf;
  const R* __restrict__ Pf;
  R* __restrict__ mo;
  R* __restrict__ Po;
  const TvModel<R> tvm;
  KF_DEV TwoFilterPipe(const ScanArgs<R>& a_, const IO<R>& io_, const TvModel<R>& tv_)
      : a(a_), io(io_), tvm(tv_) {}
  KF_DEV void bind(const SeqInfo& s, long t, int tid) {
    T = s.T;
    const long tt = s.ntiles - 1 - t;
    k0 = tt * (long)(L * blockDim.x) + (long)(blockDim.x - 1 - tid) * L;
    cst = io.cst + s.model * a.cst_stride;
    y = io.y + s.row0 * M;
    mf = io.m_in + s.row0 * N;
    Pf = io.P_in + s.row0 * N * N;
    mo = io.m_out + s.row0 * N;
    Po = io.P_out + s.row0 * N * N;
  }
  KF_DEV E op(const E& p, const E& q) const { return fcombine<N, P>(q, p); }
  // measurement of the element at row k: y_{k+2} (row k+1); none at k = T-1
  KF_DEV void load_y(long k, R (&yk)[M]) const {
#pragma unroll
    for (int c = 0; c < M; ++c) yk[c] = (k >= 0 && k + 1 < T) ? y[(k + 1) * M + c] : R(0);
  }
  KF_DEV E element(long k, const R (&yk)[M]) const {
    if constexpr (TV) {
      E e;
      if (k == T - 1) set_identity(e);
      else e = filter_element_tv<N, M, P>(tvm, k + 1, yk);
      return e;
    } else {
      return tf_element<N, M, R>(cst, T, k, yk);
    }
  }
  // With TI, a thread whose rows all hold generic elements (no row T-1) folds
  // them as the time-invariant filter does: the aggregate of L consecutive
  // generic elements has the matrix part SL and the vector part
  // b = sum_i PHI[i] y_i, eta = sum_i PSI[i] y_i (second table set, for this L).
  KF_DEV E fold() const {
    if (TI && !TV && k0 + L - 1 <= T - 2) {
      using LY = CLB<N, M, L>;
      R yv[L][M];
#pragma unroll
      for (int i = 0; i < L; ++i)
#pragma unroll
        for (int c = 0; c < M; ++c) yv[i][c] = y[(k0 + 1 + i) * M + c];
      E e;
#pragma unroll
      for (int r = 0; r < N; ++r) {
        R b = R(0), h = R(0);
#pragma unroll
        for (int i = 0; i < L; ++i)
#pragma unroll
          for (int q = 0; q < M; ++q) {
            b += cst[LY::PHI + i * N * M + r * M + q] * yv[i][q];
            h += cst[LY::PSI + i * N * M + r * M + q] * yv[i][q];
          }
        e.b[r] = b;
        e.e[r] = h;
#pragma unroll
        for (int j = 0; j < N; ++j) {
          e.A[r][j] = cst[LY::SL + r * N + j];
          e.C[r][j] = cst[LY::SL + N * N + r * N + j];
          e.J[r][j] = cst[LY::SL + 2 * N * N + r * N + j];
        }
      }
      return e;
    }
    E agg;
    set_identity(agg);
    R yn[M];
    load_y(k0 + L - 1, yn);
#pragma unroll 1
    for (int i = L - 1; i >= 0; --i) {
      const long k = k0 + i;
      R yk[M];
      copy_vec<M, R>(yn, yk);
      load_y(k - 1, yn);
      if (k < T) agg = fcombine<N, P>(element(k, yk), agg);
    }
    return agg;
  }
  KF_DEV void apply(St<N, R>& st, const E& e) const { fapply_back<N, P>(e, st.v, st.m); }
  KF_DEV void initial(St<N, R>& st) const { st_zero(st); }
  KF_DEV void anchor(const E& e, St<N, R>& st) const {
    copy_vec<N, R>(e.e, st.v);
    copy_mat<N, N, R>(e.J, st.m);
  }
  // only (eta, J) of an anchored suffix is ever read: it is the right operand
  // of every combine it takes part in
  KF_DEV void expand(const St<N, R>& st, E& v) const {
    set_identity(v);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      v.e[i] = st.v[i];
#pragma unroll
      for (int j = 0; j < N; ++j) v.J[i][j] = st.m[i][j];
    }
  }
  KF_DEV void load_f(long k, R (&x)[N], R (&Pk)[N][N]) const {
    if (k >= 0 && k < T) load_state<N, R>(mf, Pf, k, x, Pk);
  }
  KF_DEV void steps(St<N, R>& st, bool) const {
    R yn[M], xn[N], Pn[N][N];
    load_y(k0 + L - 1, yn);
    load_f(k0 + L - 1, xn, Pn);
#pragma unroll 1
    for (int i = L - 1; i >= 0; --i) {
      const long k = k0 + i;
      R yk[M], xf[N], Pk[N][N];
      copy_vec<M, R>(yn, yk);
      copy_vec<N, R>(xn, xf);
      copy_mat<N, N, R>(Pn, Pk);
      load_y(k - 1, yn);
      load_f(k - 1, xn, Pn);
      if (k >= T) continue;
      fapply_back<N, P>(element(k, yk), st.v, st.m);
      R xs[N], Ps[N][N];
      tf_combine<N, P>(xf, Pk, st.v, st.m, xs, Ps);
#pragma unroll
      for (int r = 0; r < N; ++r) {
        st_out(&mo[k * N + r], xs[r]);
#pragma unroll
        for (int c = 0; c < N; ++c) st_out(&Po[k * N * N + r * N + c], Ps[r][c]);
      }
    }
  }
};

template <int N, int M, class P, int BLOCK, int L, bool TI, bool TV = false>
__global__ __launch_bounds__(BLOCK) void k_twofilter(ScanArgs<typename P::R> a,
                                                     TvModel<typename P::R> tv,
                                                     KFS_IO_PARAMS(typename P::R)) {
  KFS_IO_MAKE(typename P::R);
  TwoFilterPipe<N, M, P, L, TI, TV> pp(a, io, tv);
  scan_tile<TwoFilterPipe<N, M, P, L, TI, TV>, N, typename P::R, BLOCK, L>(pp, a);
}

}  // namespace kfs
