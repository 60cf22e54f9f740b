// Device kernels of the open-boundary matching step (Sec. 3B, Eqs. 18-24) and
// of the Fisher-Lee transmission (Sec. 2B, Eqs. 14-16).
//
// Inputs per energy Z_k: the unperturbed Green's function on an index list
// (left boundary block, right boundary block, optional extra rows), stored
// column-major as the solver writes it, and the two lead self-energies.  With
// b = both boundary blocks (n = 2M rows) and Sigma_b = diag(Sigma_L, Sigma_R),
// the perturbed function on the boundary rows solves
//     (I - G_bb Sigma_b) G_T(b, :) = G(b, :)                        (Eq. 18 on rows b)
// and the extra rows follow as
//     G_T(l, :) = G(l, :) + G(l, b) Sigma_b G_T(b, :).               (Eq. 18 on rows l)
// Eqs. 19-24 are the two-by-two block elimination of the first system; here it
// is solved as one n x n system by blocked Gauss-Jordan elimination with
// partial pivoting, all energies in one grid.
//
// Every matrix is complex128 (double2: re, im), column-major: element (r, c)
// of a matrix with leading dimension ld is at r + ld * c.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace scocg {
namespace obm {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return {fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)};
}
__device__ __forceinline__ double2 cconj(double2 a) { return {a.x, -a.y}; }
// acc += a * b
__device__ __forceinline__ void cfma(double2& acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// One product of a batch: C = beta C + alpha op(A) B.
struct GemmPtrs {
  const double2* A;
  const double2* B;
  double2* C;
};

constexpr int GT = 64;   // output tile (rows and columns)
constexpr int GKC = 16;  // contraction chunk staged in LDS

// Batched complex GEMM, 256 threads, a 64 x 64 output tile per workgroup and
// 4 x 4 outputs per thread.  op(A) = A (m x k, leading dimension lda) or, with
// CONJ_A, A^H where A is stored k x m.  B is k x n (ldb), C is m x n (ldc).
// beta_zero skips the read of C (it may hold anything).  grid.z = batch entry.
template <bool CONJ_A>
__global__ __launch_bounds__(256) void k_zgemm(const GemmPtrs* __restrict__ list, int m, int n,
                                               int kdim, int lda, int ldb, int ldc, double2 alpha,
                                               double2 beta, int beta_zero) {
  const GemmPtrs g = list[blockIdx.z];
  __shared__ double2 As[GKC][GT + 1];
  __shared__ double2 Bs[GKC][GT + 1];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int r0 = blockIdx.x * GT, c0 = blockIdx.y * GT;
  double2 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = {0.0, 0.0};

  for (int k0 = 0; k0 < kdim; k0 += GKC) {
#pragma unroll
    for (int e = tid; e < GT * GKC; e += 256) {
      int row, kk;
      if (CONJ_A) {
        kk = e & (GKC - 1);
        row = e / GKC;
      } else {
        row = e & (GT - 1);
        kk = e / GT;
      }
      const int gr = r0 + row, gk = k0 + kk;
      double2 v = {0.0, 0.0};
      if (gr < m && gk < kdim)
        v = CONJ_A ? cconj(g.A[gk + (size_t)lda * gr]) : g.A[gr + (size_t)lda * gk];
      As[kk][row] = v;
    }
#pragma unroll
    for (int e = tid; e < GT * GKC; e += 256) {
      const int kk = e & (GKC - 1), col = e / GKC;
      const int gk = k0 + kk, gc = c0 + col;
      double2 v = {0.0, 0.0};
      if (gk < kdim && gc < n) v = g.B[gk + (size_t)ldb * gc];
      Bs[kk][col] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < GKC; ++kk) {
      double2 a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][tx + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][ty + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) cfma(acc[i][j], a[i], b[j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = c0 + ty + 16 * j;
    if (c >= n) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = r0 + tx + 16 * i;
      if (r >= m) continue;
      double2* dst = g.C + r + (size_t)ldc * c;
      double2 v = cmul(alpha, acc[i][j]);
      if (!beta_zero) v = cadd(v, cmul(beta, *dst));
      *dst = v;
    }
  }
}

// W_k = [ I_n | G_k(0:n, 0:D) ]: the augmented system of energy k, n x (n + D),
// leading dimension n.  g is [K][D][D] (column-major per energy).
// grid = (columns of W, row chunks, energies) here and in k_obm_out, k_gamma.
__global__ __launch_bounds__(256) void k_obm_init(const double2* __restrict__ g, double2* W,
                                                  int n, int D) {
  const int k = blockIdx.z;
  const int c = blockIdx.x;  // column of W, 0 .. n + D - 1
  const double2* gk = g + (size_t)k * D * D;
  double2* Wc = W + (size_t)k * n * (n + D) + (size_t)n * c;
  for (int i = blockIdx.y * 256 + threadIdx.x; i < n; i += gridDim.y * 256) {
    double2 v;
    if (c < n)
      v = {i == c ? 1.0 : 0.0, 0.0};
    else
      v = gk[i + (size_t)D * (c - n)];
    Wc[i] = v;
  }
}

// Blocked Gauss-Jordan elimination with partial pivoting on W_k = [A | RHS]
// (n x ncol, leading dimension n), panels of GJ_W pivot columns.
//
// Panel kernel (one workgroup per energy) for pivots j = j0 .. j0+w-1: pick
// p = argmax_{i >= j} |W(i, j)| (smallest i on ties), swap rows j and p over
// every column from j on (so the columns right of the panel already hold
// their final row order) and over the multipliers of the earlier pivots of
// the panel, keep the pivot value and the multipliers f^(j)_i = W(i, j)
// (i != j; f^(j)_j = 0), and eliminate inside the panel columns only.
//
// Columns right of the panel: with v_J the rows j0.. of a column and F the
// panel's multipliers, the panel's w eliminations amount to
//   z_j = (v_j - sum_{j' < j} f^(j')_j z_j') / pivot_j          (forward sweep)
//   new v_j = z_j - sum_{j' > j} f^(j')_j z_j'                   (rows j of the panel)
//   new v_i = v_i - sum_j' f^(j')_i z_j'                         (every other row)
// The panel kernel snapshots v_J (Vj) as each row settles, the sweep kernel turns
// it into z in place, and the update kernel applies the last two lines by 64 x 64
// tiles, so each element is read and written once per panel instead of once per
// pivot.  A zero or non-finite pivot marks the energy failed; later kernels skip it.
constexpr int GJ_W = 32;     // pivots per panel
constexpr int GJ_EB = 8;     // panel columns of a row loaded together in the elimination
// threads of the panel kernel: 512, or 1024 above n = 1024 rows (chosen at launch)

// Vj [K][GJ_W][ncol]: row j0 + jj of every column right of the panel, as it stands
// once its swap is done (its final row order); the sweep and update read it from
// here, so the tile that owns the panel rows can overwrite them in W.
template <int GJ_PNT>
__global__ __launch_bounds__(GJ_PNT) void k_gj_panel(double2* W, double2* F, double2* pivv,
                                                     double2* Vj, int32_t* fail, int n,
                                                     int ncol, int j0, int w) {
  const int k = blockIdx.x;
  if (fail[k]) return;
  double2* Wk = W + (size_t)k * n * ncol;
  double2* Fk = F + (size_t)k * n * GJ_W;
  __shared__ double s_val[GJ_PNT / 64];
  __shared__ int s_idx[GJ_PNT / 64];
  __shared__ double2 s_prow[GJ_W];  // row j over the panel columns, after the swap
  const int tid = threadIdx.x;
  const int jend = j0 + w;
  // pivot candidates of the first column; later columns' candidates are taken while
  // the previous pivot is eliminated
  double best = -1.0;
  int bi = n;
  for (int i = j0 + tid; i < n; i += GJ_PNT) {
    const double a = cabs2(Wk[i + (size_t)n * j0]);
    if (a > best) {  // strict: the smallest index of this thread's rows on ties
      best = a;
      bi = i;
    }
  }
  constexpr int NWAVE = GJ_PNT / 64;
  for (int jj = 0; jj < w; ++jj) {
    const int j = j0 + jj;
    // argmax (largest |W(i, j)|^2, smallest i on ties): across the 64 lanes of each
    // wave by shuffles, then across the waves in LDS
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(best, off);
      const int oi = __shfl_xor(bi, off);
      if (o > best || (o == best && oi < bi)) {
        best = o;
        bi = oi;
      }
    }
    if ((tid & 63) == 0) {
      s_val[tid >> 6] = best;
      s_idx[tid >> 6] = bi;
    }
    __syncthreads();
    double pv = s_val[0];
    int p = s_idx[0];
#pragma unroll
    for (int q = 1; q < NWAVE; ++q) {
      const double o = s_val[q];
      const int oi = s_idx[q];
      if (o > pv || (o == pv && oi < p)) {
        pv = o;
        p = oi;
      }
    }
    if (!(pv > 0.0) || !isfinite(pv) || p >= n) {
      if (tid == 0) fail[k] = 1;
      return;
    }
    // swap rows j and p from column j on; the threads of the panel columns keep the
    // new row j for everyone
    for (int c = j + tid; c < ncol; c += GJ_PNT) {
      double2* a = Wk + j + (size_t)n * c;
      double2 v = *a;
      if (p != j) {
        double2* b = Wk + p + (size_t)n * c;
        const double2 t = v;
        v = *b;
        *a = v;
        *b = t;
      }
      if (c < jend)
        s_prow[c - j0] = v;
      else
        Vj[((size_t)k * GJ_W + jj) * ncol + c] = v;
    }
    if (p != j)
      for (int c = tid; c < jj; c += GJ_PNT) {
        double2* a = Fk + j + (size_t)n * c;
        double2* b = Fk + p + (size_t)n * c;
        const double2 t = *a;
        *a = *b;
        *b = t;
      }
    __syncthreads();
    const double2 piv = s_prow[jj];
    const double inv_den = 1.0 / cabs2(piv);
    const double2 inv = {piv.x * inv_den, -piv.y * inv_den};
    if (tid == 0) pivv[(size_t)k * GJ_W + jj] = piv;
    // every row i: multiplier f_i = W(i, j) (0 for i = j), then the panel columns
    // right of j: row j scaled by 1/pivot, other rows minus f_i times that
    best = -1.0;
    bi = n;
    for (int i = tid; i < n; i += GJ_PNT) {
      const double2 fi = (i == j) ? double2{0.0, 0.0} : Wk[i + (size_t)n * j];
      Fk[i + (size_t)n * jj] = fi;
      // the row's panel columns in batches of GJ_EB: all loads of a batch are issued
      // before its first store, so a row costs a few memory round trips, not one per
      // column
      for (int cb = j + 1; cb < jend; cb += GJ_EB) {
        double2 v[GJ_EB];
#pragma unroll
        for (int q = 0; q < GJ_EB; ++q)
          v[q] = (cb + q < jend && i != j) ? Wk[i + (size_t)n * (cb + q)] : double2{0.0, 0.0};
#pragma unroll
        for (int q = 0; q < GJ_EB; ++q) {
          const int c = cb + q;
          if (c >= jend) continue;
          const double2 pj = cmul(s_prow[c - j0], inv);
          double2 r;
          if (i == j) {
            r = pj;
          } else {
            r = v[q];
            r.x = fma(-fi.x, pj.x, fma(fi.y, pj.y, r.x));
            r.y = fma(-fi.x, pj.y, fma(-fi.y, pj.x, r.y));
          }
          Wk[i + (size_t)n * c] = r;
          if (c == j + 1 && i > j) {
            const double m = cabs2(r);
            if (m > best) {
              best = m;
              bi = i;
            }
          }
        }
      }
    }
    __syncthreads();  // s_prow, s_val and this step's writes are settled before the next step
  }
}

// Forward sweep of the panel rows of every column right of the panel, in place in
// Vj (one thread per column; the subtractions of each z_j in the order j' = 0, 1, ...
// of the elimination):
//   z_j = (v_j - sum_{j' < j} f^(j')_j z_j') / pivot_j
// grid = (column groups of 64 over columns j0+w .. ncol-1, energies), 64 threads.
__global__ __launch_bounds__(64) void k_gj_sweep(double2* Vj, const double2* __restrict__ F,
                                                 const double2* __restrict__ pivv,
                                                 const int32_t* __restrict__ fail, int n,
                                                 int ncol, int j0, int w) {
  const int k = blockIdx.y;
  if (fail[k]) return;
  __shared__ double2 fj[GJ_W][GJ_W + 1];  // fj[i][j'] = f^(j')_{j0+i}
  __shared__ double2 pinv[GJ_W];
  const double2* Fk = F + (size_t)k * n * GJ_W;
  const int tid = threadIdx.x;
  for (int e = tid; e < w * w; e += 64) {
    const int i = e % w, jp = e / w;
    fj[i][jp] = Fk[(j0 + i) + (size_t)n * jp];
  }
  if (tid < w) {
    const double2 pv = pivv[(size_t)k * GJ_W + tid];
    const double d = 1.0 / cabs2(pv);
    pinv[tid] = {pv.x * d, -pv.y * d};
  }
  __syncthreads();
  const int c = j0 + w + blockIdx.x * 64 + tid;
  if (c >= ncol) return;
  double2* col = Vj + (size_t)k * GJ_W * ncol + c;
  double2 z[GJ_W];
#pragma unroll
  for (int jj = 0; jj < GJ_W; ++jj) z[jj] = jj < w ? col[(size_t)jj * ncol] : double2{0.0, 0.0};
#pragma unroll
  for (int jj = 0; jj < GJ_W; ++jj) {
    if (jj < w) {  // a predicate, not a break: every index of z stays a constant
      double2 v = z[jj];
#pragma unroll
      for (int jp = 0; jp < jj; ++jp) {
        const double2 f = fj[jj][jp];
        v.x = fma(-f.x, z[jp].x, fma(f.y, z[jp].y, v.x));
        v.y = fma(-f.x, z[jp].y, fma(-f.y, z[jp].x, v.y));
      }
      z[jj] = cmul(v, pinv[jj]);
      col[(size_t)jj * ncol] = z[jj];
    }
  }
}

// Update of the columns right of the panel as a tiled product: workgroup (column tile,
// row tile, energy) owns a GJ_T x GJ_T tile of W.  The swept panel rows z of its
// columns (Vj) and the multiplier rows of its tile pass through LDS GJ_KC pivots at a
// time (34 KB, so that four workgroups share a CU and one's loads overlap another's
// arithmetic) -- the lower multipliers of the panel rows zeroed, so those rows start
// from z and take only the upper terms -- and each thread updates 4 x 4 elements:
//   rows of the panel:  z_j - sum_{j' > j} f^(j')_j z_j';   other rows:  v_i - sum_j' f^(j')_i z_j'.
// Subtracting a zeroed term leaves a finite value bit for bit unchanged, so this equals
// the row-by-row update.  (The same product on the FP64 matrix cores,
// v_mfma_f64_16x16x4f64, was slower here: their peak on this chip is the vector peak,
// and the 64 KB of operands per workgroup halved the workgroups per CU.)
constexpr int GJ_T = 64;   // rows and columns per workgroup tile of the update
constexpr int GJ_KC = 16;  // pivots per LDS stage of the update

__global__ __launch_bounds__(256) void k_gj_update(double2* W, const double2* __restrict__ F,
                                                   const double2* __restrict__ Vj,
                                                   const int32_t* __restrict__ fail, int n,
                                                   int ncol, int j0, int w) {
  const int k = blockIdx.z;
  if (fail[k]) return;
  const int c0 = j0 + w + blockIdx.x * GJ_T;
  const int r0 = blockIdx.y * GJ_T;
  if (c0 >= ncol || r0 >= n) return;
  double2* Wk = W + (size_t)k * n * ncol;
  const double2* Fk = F + (size_t)k * n * GJ_W;
  const double2* Vk = Vj + (size_t)k * GJ_W * ncol;
  __shared__ double2 zs[GJ_KC][GJ_T + 1];  // swept panel rows kc.. of the tile's columns
  __shared__ double2 fs[GJ_T][GJ_KC + 1];  // multipliers kc.. of the tile's rows
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  double2 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = r0 + tx + 16 * a;
    const bool in_panel = i >= j0 && i < j0 + w;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int c = c0 + ty + 16 * b;
      acc[a][b] = (i >= n || c >= ncol) ? double2{0.0, 0.0}
                  : (in_panel ? Vk[(size_t)(i - j0) * ncol + c] : Wk[i + (size_t)n * c]);
    }
  }
  for (int kc = 0; kc < w; kc += GJ_KC) {
    const int kw = min(GJ_KC, w - kc);
    if (kc > 0) __syncthreads();  // the previous stage's readers are done
    for (int e = tid; e < kw * GJ_T; e += 256) {
      const int c = e % GJ_T, i = e / GJ_T;
      zs[i][c] = c0 + c < ncol ? Vk[(size_t)(kc + i) * ncol + c0 + c] : double2{0.0, 0.0};
    }
    for (int e = tid; e < GJ_T * kw; e += 256) {
      const int r = e % GJ_T, jq = e / GJ_T, jp = kc + jq;
      const int i = r0 + r;
      double2 f = {0.0, 0.0};
      // panel rows take only the multipliers of later pivots
      if (i < n && !(i >= j0 && i < j0 + w && jp <= i - j0)) f = Fk[i + (size_t)n * jp];
      fs[r][jq] = f;
    }
    __syncthreads();
    for (int jq = 0; jq < kw; ++jq) {
      double2 f[4], z[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) f[a] = fs[tx + 16 * a][jq];
#pragma unroll
      for (int b = 0; b < 4; ++b) z[b] = zs[jq][ty + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          acc[a][b].x = fma(-f[a].x, z[b].x, fma(f[a].y, z[b].y, acc[a][b].x));
          acc[a][b].y = fma(-f[a].x, z[b].y, fma(-f[a].y, z[b].x, acc[a][b].y));
        }
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = r0 + tx + 16 * a;
    if (i >= n) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int c = c0 + ty + 16 * b;
      if (c < ncol) Wk[i + (size_t)n * c] = acc[a][b];
    }
  }
}

// G_T rows: rows 0..n-1 from the solved system (W columns n..n+D-1), rows
// n..D-1 start as the unperturbed rows (the extra-row update adds to them).  An
// energy whose elimination met a zero pivot gets NaN in every row, so the
// extra-row update that follows (an addition to these rows) leaves NaN too.
__global__ __launch_bounds__(256) void k_obm_out(const double2* __restrict__ W,
                                                 const double2* __restrict__ g, double2* gt,
                                                 const int32_t* __restrict__ fail, int n, int D) {
  const int k = blockIdx.z;
  const int c = blockIdx.x;
  const bool bad = fail[k] != 0;
  const double2* Wk = W + (size_t)k * n * (n + D) + (size_t)n * (n + c);
  const double2* gk = g + (size_t)k * D * D + (size_t)D * c;
  double2* out = gt + (size_t)k * D * D + (size_t)D * c;
  for (int i = blockIdx.y * 256 + threadIdx.x; i < D; i += gridDim.y * 256)
    out[i] = bad ? double2{NAN, NAN} : (i < n ? Wk[i] : gk[i]);
}

// Gamma = i (Sigma - Sigma^H) (Eq. 16), M x M per energy.
__global__ __launch_bounds__(256) void k_gamma(const double2* __restrict__ sig, double2* gam,
                                               int M) {
  const int k = blockIdx.z;
  const int c = blockIdx.x;
  const double2* s = sig + (size_t)k * M * M;
  double2* o = gam + (size_t)k * M * M + (size_t)M * c;
  for (int r = blockIdx.y * 256 + threadIdx.x; r < M; r += gridDim.y * 256) {
    const double2 a = s[r + (size_t)M * c];
    const double2 b = s[c + (size_t)M * r];
    // i * (a - conj(b))
    const double2 d = {a.x - b.x, a.y + b.y};
    o[r] = {-d.y, d.x};
  }
}

// T_k = sum_{a, c} Gamma_L(a, c) Q(c, a) with Q = Y^H Gamma_R Y and
// Y = G_T(right block, left block): the trace of Eq. 14.  Gamma_L is formed on
// the fly from Sigma_L.  One workgroup per energy, fixed summation order.
__global__ __launch_bounds__(256) void k_trace_gamma(const double2* __restrict__ sig_l,
                                                     const double2* __restrict__ Q, double2* T,
                                                     const int32_t* __restrict__ fail, int M) {
  const int k = blockIdx.x;
  const double2* s = sig_l + (size_t)k * M * M;
  const double2* q = Q + (size_t)k * M * M;
  __shared__ double sx[256], sy[256];
  const int tid = threadIdx.x;
  double2 acc = {0.0, 0.0};
  const int64_t MM = (int64_t)M * M;
  for (int64_t e = tid; e < MM; e += 256) {
    const int a = (int)(e % M), c = (int)(e / M);
    const double2 sa = s[a + (size_t)M * c];
    const double2 sb = s[c + (size_t)M * a];
    const double2 d = {sa.x - sb.x, sa.y + sb.y};
    const double2 gl = {-d.y, d.x};
    cfma(acc, gl, q[c + (size_t)M * a]);
  }
  sx[tid] = acc.x;
  sy[tid] = acc.y;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) {
      sx[tid] += sx[tid + st];
      sy[tid] += sy[tid + st];
    }
    __syncthreads();
  }
  if (tid == 0) T[k] = fail[k] ? double2{NAN, NAN} : double2{sx[0], sy[0]};
}

// DOS_k = -Im sum_{i < L} G_T(n + i, n + i) / pi over the extra rows.
__global__ __launch_bounds__(256) void k_dos(const double2* __restrict__ gt, double* dos,
                                             const int32_t* __restrict__ fail, int n, int D,
                                             int L) {
  const int k = blockIdx.x;
  const double2* gk = gt + (size_t)k * D * D;
  __shared__ double sy[256];
  const int tid = threadIdx.x;
  double acc = 0.0;
  for (int i = tid; i < L; i += 256) acc += gk[(n + i) + (size_t)D * (n + i)].y;
  sy[tid] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) sy[tid] += sy[tid + st];
    __syncthreads();
  }
  if (tid == 0) dos[k] = fail[k] ? NAN : -sy[0] / M_PI;
}

}  // namespace obm
}  // namespace scocg
