// Device kernels of the shifted COCG solver (gfx950).
//
// Data layout in HBM (B = columns per block, 8 for complex128, 16 for complex64,
// so one grid point of one block is 128 contiguous bytes):
//   Krylov vectors      [nb][N][B]        complex<T>   (RHS innermost)
//   shift vectors x, p  [nb][K][nS][B]    x complex128, p complex<T>
//   shift state         [nb][K][B]        ShiftState (pi_{n-1}, pi_n, status)
//   column state        [nb*B]            ColState (seed scalars, FP64)
// Per seed iteration n the host enqueues:
//   k_proj      C_a = D_a P_a^T r_n for every atom                    (nonlocal part of H)
//   k_stencil<MU>     partials of mu_n = (r_n, A r_n),  A = z_s - H    (Eq. A5 numerator terms)
//   k_alpha     alpha_n, c_n = beta_{n-1} alpha_n / alpha_{n-1}       (Eq. A5)
//   k_stencil<UPDATE> r_{n+1} = (1+c_n) r_n - alpha_n A r_n - c_n r_{n-1}  (Eq. A3), in place
//                     over r_{n-1}; partials of rho_{n+1}, ||r_{n+1}||^2
//   k_control   beta_n (Eq. A6); pi, alpha^(i), beta^(i) per shift (Eqs. A8-A10);
//               convergence, compaction of active shifts; seed switch (Eq. A13)
//   k_shift     x^(i), p^(i) on the rows S (Eqs. A11-A12 with Eq. A7)
// A r_n is recomputed in the UPDATE pass instead of being stored, so one
// iteration streams r_n twice, r_{n-1} once and writes r_{n+1} once.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scocg {

constexpr int WG = 256;  // threads per workgroup for the streaming kernels

// ------------------------------------------------------------------ complex helpers
template <typename T> struct cplx_of;
template <> struct cplx_of<double> { using type = double2; };
template <> struct cplx_of<float> { using type = float2; };

__host__ __device__ __forceinline__ double2 mk(double a, double b) { return make_double2(a, b); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return mk(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return mk(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  // Smith's algorithm: avoids overflow of |b|^2 for large pi values
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, d = b.x + b.y * r;
    return mk((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  }
  double r = b.x / b.y, d = b.y + b.x * r;
  return mk((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ double cabsd(double2 a) { return hypot(a.x, a.y); }
__device__ __forceinline__ bool cfinite(double2 a) { return isfinite(a.x) && isfinite(a.y); }

__device__ __forceinline__ double2 to_d(double2 a) { return a; }
__device__ __forceinline__ double2 to_d(float2 a) { return mk(a.x, a.y); }
template <typename V> __device__ __forceinline__ V from_d(double2 a);
template <> __device__ __forceinline__ double2 from_d<double2>(double2 a) { return a; }
template <> __device__ __forceinline__ float2 from_d<float2>(double2 a) {
  return make_float2((float)a.x, (float)a.y);
}

// ------------------------------------------------------------------ state records
struct ColState {
  double2 rho;         // (r_n, r_n) of the current seed (unscaled true value)
  double2 alpha_prev;  // alpha_{n-1}
  double2 beta_prev;   // beta_{n-1}
  double2 alpha;       // alpha_n (set by k_alpha)
  double2 c;           // beta_{n-1} alpha_n / alpha_{n-1}
  double2 zs;          // current seed energy
  double2 scale[2];    // stored Krylov buffer b holds r / scale[b] (lazy seed-switch rescale)
  double2 ar, aw, ap;  // r_{n+1} = ar r^st_n + aw (A r^st_n) + ap r^st_{n-1}
  double bnorm;        // ||b||
  int32_t seed;        // seed shift index
  int32_t done;        // column finished
  int32_t breakdown;   // column hit a vanishing bilinear form
  int32_t nswitch;     // seed switches so far
  int32_t iters;       // seed iterations done
  int32_t pad_;
};

struct ShiftState {
  double2 pi_prev;  // pi_{n-1}
  double2 pi;       // pi_n
  double est;       // ||r_n|| / |pi_n| / ||b||
  int32_t iters;    // iteration at which the pair froze
  int32_t status;   // 0 converged, 1 max-iter, 2 breakdown, 3 unused column
  int32_t active;   // still iterating
  int32_t pad_;
};

struct ShiftCoef {
  double2 a;   // alpha^(i)_n
  double2 b;   // beta^(i)_n
  double2 f;   // 1 / pi_{n+1} times the stored-buffer scale
  int32_t upd; // 1: apply this iteration
  int32_t pad_[3];
};

enum { ST_CONVERGED = 0, ST_MAXITER = 1, ST_BREAKDOWN = 2, ST_UNUSED = 3 };

// Real stencil coefficients, by value in the kernel argument segment.
template <typename T> struct Coefs {
  T cx[5], cy[5], cz[5];
  T c0;  // cx[0] + cy[0] + cz[0]
};

// ------------------------------------------------------------------ stencil pass
enum { MODE_MU = 0, MODE_UPDATE = 1, MODE_APPLY = 2 };

template <typename T>
struct StencilArgs {
  using cT = typename cplx_of<T>::type;
  const cT* r;           // [nb][N][B] stored r_n
  cT* io;                // UPDATE: r_{n-1} in, r_{n+1} out; APPLY: H r out
  const T* vloc;         // [N]
  Coefs<T> co;
  int nx, ny, nz, nxy;
  int zc;                // planes per workgroup
  const int32_t* prow;   // [N+1] point -> projector entries (null if no atoms)
  const int32_t* patom;  // [E] atom of each entry
  const T* pval;         // [E][4] projector values
  const cT* dc;          // [nb][n_atoms][4][B] D_a P_a^T r
  int n_atoms;
  const ColState* cols;  // [nb*B]
  const int32_t* blk_active;  // [nb] (null: all active)
  double2* part0;        // [nb][n_wg][B] mu or rho partials
  double* part1;         // [nb][n_wg][B] ||r||^2 partials (UPDATE)
};

// One thread owns one (x-y point, column) and marches along z over zc planes
// with a register queue of the 2*NF+1 z-neighbours; x and y neighbours are
// read through L1/L2.  Workgroup reductions of the dot partials are in a
// fixed tree order (bitwise repeatable, no atomics).
template <typename T, int NF, int B, int MODE>
__global__ __launch_bounds__(WG) void k_stencil(StencilArgs<T> a) {
  using cT = typename cplx_of<T>::type;
  constexpr int PTS = WG / B;
  const int tid = threadIdx.x;
  const int c = tid % B;
  const int pl = tid / B;
  const int cb = blockIdx.z;
  if (a.blk_active && !a.blk_active[cb]) return;
  const int q = blockIdx.x * PTS + pl;
  const bool valid = q < a.nxy;
  const int z0 = blockIdx.y * a.zc;
  const int z1 = min(z0 + a.zc, a.nz);
  const int64_t N = (int64_t)a.nxy * a.nz;
  const cT* rb = a.r + (int64_t)cb * N * B + c;
  const int j = cb * B + c;

  int xo_p[NF + 1], xo_m[NF + 1], yo_p[NF + 1], yo_m[NF + 1];
  {
    const int qq = valid ? q : 0;
    const int ix = qq % a.nx, iy = qq / a.nx;
#pragma unroll
    for (int k = 1; k <= NF; ++k) {
      int xp = ix + k; if (xp >= a.nx) xp -= a.nx;
      int xm = ix - k; if (xm < 0) xm += a.nx;
      int yp = iy + k; if (yp >= a.ny) yp -= a.ny;
      int ym = iy - k; if (ym < 0) ym += a.ny;
      xo_p[k] = xp + iy * a.nx;
      xo_m[k] = xm + iy * a.nx;
      yo_p[k] = ix + yp * a.nx;
      yo_m[k] = ix + ym * a.nx;
    }
  }
  double2 zs = mk(0, 0), ar = mk(0, 0), aw = mk(0, 0), ap = mk(0, 0);
  if (MODE != MODE_APPLY) {
    const ColState& cs = a.cols[j];
    zs = cs.zs;
    ar = cs.ar; aw = cs.aw; ap = cs.ap;
  }
  const T zr = (T)zs.x, zi = (T)zs.y;

  cT Q[2 * NF + 1];
#pragma unroll
  for (int d = 0; d < 2 * NF; ++d) {
    const int iz = z0 - NF + d;
    Q[d] = (valid && iz >= 0 && iz < a.nz) ? rb[((int64_t)iz * a.nxy + q) * B] : cT{0, 0};
  }
  double2 acc0 = mk(0, 0);
  double acc1 = 0.0;
  for (int iz = z0; iz < z1; ++iz) {
    {
      const int izn = iz + NF;
      Q[2 * NF] = (valid && izn < a.nz) ? rb[((int64_t)izn * a.nxy + q) * B] : cT{0, 0};
    }
    if (valid) {
      const int64_t pbase = (int64_t)iz * a.nxy;
      const int64_t p = pbase + q;
      const cT ctr = Q[NF];
      const T dg = a.co.c0 + a.vloc[p];
      T hr = dg * ctr.x, hi = dg * ctr.y;
#pragma unroll
      for (int k = 1; k <= NF; ++k) {
        const cT zp = Q[NF + k], zm = Q[NF - k];
        const cT xp = rb[(pbase + xo_p[k]) * B], xm = rb[(pbase + xo_m[k]) * B];
        const cT yp = rb[(pbase + yo_p[k]) * B], ym = rb[(pbase + yo_m[k]) * B];
        hr += a.co.cz[k] * (zp.x + zm.x) + a.co.cx[k] * (xp.x + xm.x) + a.co.cy[k] * (yp.x + ym.x);
        hi += a.co.cz[k] * (zp.y + zm.y) + a.co.cx[k] * (xp.y + xm.y) + a.co.cy[k] * (yp.y + ym.y);
      }
      if (a.prow) {
        const int e0 = a.prow[p], e1 = a.prow[p + 1];
        for (int e = e0; e < e1; ++e) {
          const cT* dca = a.dc + ((int64_t)cb * a.n_atoms + a.patom[e]) * 4 * B + c;
          const T* pv = a.pval + (int64_t)e * 4;
#pragma unroll
          for (int l = 0; l < 4; ++l) {
            const cT d = dca[l * B];
            hr += pv[l] * d.x;
            hi += pv[l] * d.y;
          }
        }
      }
      if (MODE == MODE_APPLY) {
        cT o; o.x = hr; o.y = hi;
        a.io[(p * B) + (int64_t)cb * N * B + c] = o;
      } else {
        // w = (z_s - H) r
        const T wr = zr * ctr.x - zi * ctr.y - hr;
        const T wi = zr * ctr.y + zi * ctr.x - hi;
        if (MODE == MODE_MU) {
          const double cr = ctr.x, ci = ctr.y;
          acc0.x += cr * (double)wr - ci * (double)wi;
          acc0.y += cr * (double)wi + ci * (double)wr;
        } else {
          cT* iop = a.io + (int64_t)cb * N * B + p * B + c;
          const double2 rp = to_d(*iop);
          const double2 rc = to_d(ctr);
          const double2 ww = mk(wr, wi);
          double2 rn = cmul(ar, rc);
          rn = cadd(rn, cmul(aw, ww));
          rn = cadd(rn, cmul(ap, rp));
          const cT rs = from_d<cT>(rn);
          *iop = rs;
          const double2 rq = to_d(rs);
          acc0.x += rq.x * rq.x - rq.y * rq.y;
          acc0.y += 2.0 * rq.x * rq.y;
          acc1 += rq.x * rq.x + rq.y * rq.y;
        }
      }
    }
#pragma unroll
    for (int d = 0; d < 2 * NF; ++d) Q[d] = Q[d + 1];
  }
  if (MODE == MODE_APPLY) return;

  __shared__ double2 s0[WG];
  __shared__ double s1[WG];
  s0[tid] = acc0;
  if (MODE == MODE_UPDATE) s1[tid] = acc1;
  __syncthreads();
#pragma unroll
  for (int s = PTS / 2; s >= 1; s >>= 1) {
    if (pl < s) {
      s0[tid] = cadd(s0[tid], s0[tid + s * B]);
      if (MODE == MODE_UPDATE) s1[tid] += s1[tid + s * B];
    }
    __syncthreads();
  }
  if (pl == 0) {
    const int nwg = gridDim.x * gridDim.y;
    const int wg = blockIdx.x + gridDim.x * blockIdx.y;
    const int64_t o = ((int64_t)cb * nwg + wg) * B + c;
    a.part0[o] = s0[tid];
    if (MODE == MODE_UPDATE) a.part1[o] = s1[tid];
  }
}

// ------------------------------------------------------------------ projector contraction
// dc[cb][a][l][c] = D_a[l] * sum_e P_a[e][l] r[idx_e][c], one workgroup per (atom, block).
template <typename T, int B>
__global__ __launch_bounds__(WG) void k_proj(const typename cplx_of<T>::type* __restrict__ r,
                                              int64_t N, const int32_t* __restrict__ aptr,
                                              const int32_t* __restrict__ aidx,
                                              const T* __restrict__ aval, const T* __restrict__ aD,
                                              int n_proj, int n_atoms,
                                              typename cplx_of<T>::type* __restrict__ dc,
                                              const int32_t* __restrict__ blk_active) {
  using cT = typename cplx_of<T>::type;
  constexpr int PTS = WG / B;
  const int tid = threadIdx.x, c = tid % B, ln = tid / B;
  const int at = blockIdx.x, cb = blockIdx.y;
  if (blk_active && !blk_active[cb]) return;
  const cT* rb = r + (int64_t)cb * N * B + c;
  T acc[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  const int e0 = aptr[at], e1 = aptr[at + 1];
  for (int e = e0 + ln; e < e1; e += PTS) {
    const cT v = rb[(int64_t)aidx[e] * B];
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const T pv = aval[(int64_t)e * 4 + l];
      acc[l][0] += pv * v.x;
      acc[l][1] += pv * v.y;
    }
  }
  __shared__ T sh[4][2][WG];
#pragma unroll
  for (int l = 0; l < 4; ++l) { sh[l][0][tid] = acc[l][0]; sh[l][1][tid] = acc[l][1]; }
  __syncthreads();
  for (int s = PTS / 2; s >= 1; s >>= 1) {
    if (ln < s) {
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        sh[l][0][tid] += sh[l][0][tid + s * B];
        sh[l][1][tid] += sh[l][1][tid + s * B];
      }
    }
    __syncthreads();
  }
  if (ln == 0) {
    cT* o = dc + ((int64_t)cb * n_atoms + at) * 4 * B + c;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const T d = l < n_proj ? aD[at * 4 + l] : (T)0;
      cT v; v.x = d * sh[l][0][tid]; v.y = d * sh[l][1][tid];
      o[l * B] = v;
    }
  }
}

// ------------------------------------------------------------------ seed alpha (Eq. A5)
// One workgroup per column block: fixed-order reduction of the mu partials, then
//   alpha_n = rho_n / (mu_n - beta_{n-1}/alpha_{n-1} rho_n),  c_n = beta_{n-1} alpha_n / alpha_{n-1}
// and the coefficients of the UPDATE pass in stored-buffer units.
template <int B>
__global__ __launch_bounds__(WG) void k_alpha(const double2* __restrict__ part, int nwg,
                                               ColState* __restrict__ cols, int buf_cur,
                                               const int32_t* __restrict__ blk_active) {
  constexpr int PTS = WG / B;
  const int tid = threadIdx.x, c = tid % B, ln = tid / B, cb = blockIdx.x;
  if (!blk_active[cb]) return;
  double2 acc = mk(0, 0);
  for (int w = ln; w < nwg; w += PTS) acc = cadd(acc, part[((int64_t)cb * nwg + w) * B + c]);
  __shared__ double2 sh[WG];
  sh[tid] = acc;
  __syncthreads();
  for (int s = PTS / 2; s >= 1; s >>= 1) {
    if (ln < s) sh[tid] = cadd(sh[tid], sh[tid + s * B]);
    __syncthreads();
  }
  if (ln != 0) return;
  ColState& cs = cols[cb * B + c];
  if (cs.done) {
    cs.ar = cs.aw = cs.ap = mk(0, 0);
    return;
  }
  const double2 s_cur = cs.scale[buf_cur], s_prev = cs.scale[buf_cur ^ 1];
  // stored r^st = r / s  =>  mu = s^2 mu^st (unconjugated bilinear form)
  const double2 mu = cmul(cmul(s_cur, s_cur), sh[tid]);
  const double2 denom = csub(mu, cmul(cdiv(cs.beta_prev, cs.alpha_prev), cs.rho));
  const double2 alpha = cdiv(cs.rho, denom);
  const double2 cc = cdiv(cmul(cs.beta_prev, alpha), cs.alpha_prev);
  if (!(cabs2(denom) > 0.0) || !(cabs2(cs.rho) > 0.0) || !cfinite(alpha) || !cfinite(cc)) {
    cs.breakdown = 1;
    cs.ar = cs.aw = cs.ap = mk(0, 0);
    return;
  }
  cs.alpha = alpha;
  cs.c = cc;
  cs.ar = cmul(mk(1.0 + cc.x, cc.y), s_cur);
  cs.aw = cmul(mk(-alpha.x, -alpha.y), s_cur);
  cs.ap = cmul(mk(-cc.x, -cc.y), s_prev);
}

// ------------------------------------------------------------------ column control
struct ControlArgs {
  const double2* part_rho;  // [nb][nwg][B]
  const double* part_nu;    // [nb][nwg][B]
  int nwg;
  ColState* cols;
  ShiftState* sh;           // [nb][K][B]
  ShiftCoef* coef;          // [nb][K][B]
  const double2* z;         // [nb][K][B] energies per column
  int K;
  int32_t* list;            // [2][nb][K]
  int32_t* cnt;             // [2][nb]
  int32_t* k5cnt;           // [nb] entries for k_shift this iteration
  int32_t* blk_active;      // [nb]
  int32_t* blk_iter;        // [nb]
  int par;                  // list parity of this iteration (reads list[par], writes list[par^1])
  int buf_new;              // Krylov buffer holding r_{n+1}
  double tol;
  int64_t max_iter;
  int seed_switch;
};

// One workgroup per column block (B columns x K shifts):
//   beta_n = rho_{n+1} / rho_n                                            (Eq. A6)
//   pi_{n+1} = (1 + c_n + alpha_n sigma) pi_n - c_n pi_{n-1}, sigma = z_k - z_s   (Eq. A8)
//   alpha^(k)_n = pi_n/pi_{n+1} alpha_n,  beta^(k)_n = (pi_n/pi_{n+1})^2 beta_n  (Eqs. A9-A10)
//   freeze (k, j) once ||r_{n+1}|| / |pi_{n+1}| <= tol ||b||; compact the active list;
//   seed switch to the active shift of smallest |pi_{n+1}| once the seed froze (Eq. A13).
// Thread t always serves column t % B (WG is a multiple of B), so every
// per-column reduction is one fixed-order tree over the WG/B lanes of that column.
template <int B>
__global__ __launch_bounds__(WG) void k_control(ControlArgs a) {
  constexpr int PTS = WG / B;
  const int tid = threadIdx.x, c = tid % B, ln = tid / B, cb = blockIdx.x;
  if (!a.blk_active[cb]) {
    if (tid == 0) a.k5cnt[cb] = 0;
    return;
  }
  const int K = a.K;
  const int n = a.blk_iter[cb];
  __shared__ double2 sh_rho[WG];
  __shared__ double sh_nu[WG];
  __shared__ double s_best[WG];
  __shared__ int s_bestk[WG];
  __shared__ int s_scan[WG];
  __shared__ double2 s_alpha[B], s_beta[B], s_c[B], s_zs[B], s_fn[B], s_fc[B];
  __shared__ double s_nrm[B];
  __shared__ int s_live[B], s_cnt_col[B], s_argmin[B], s_sw[B];
  __shared__ int s_total;

  // 1. reduce rho_{n+1} and ||r_{n+1}||^2 partials
  {
    double2 ra = mk(0, 0);
    double na = 0.0;
    for (int w = ln; w < a.nwg; w += PTS) {
      const int64_t o = ((int64_t)cb * a.nwg + w) * B + c;
      ra = cadd(ra, a.part_rho[o]);
      na += a.part_nu[o];
    }
    sh_rho[tid] = ra;
    sh_nu[tid] = na;
  }
  __syncthreads();
  for (int s = PTS / 2; s >= 1; s >>= 1) {
    if (ln < s) {
      sh_rho[tid] = cadd(sh_rho[tid], sh_rho[tid + s * B]);
      sh_nu[tid] += sh_nu[tid + s * B];
    }
    __syncthreads();
  }
  if (tid < B) {
    ColState& cs = a.cols[cb * B + tid];
    cs.scale[a.buf_new] = mk(1.0, 0.0);  // r_{n+1} was just written unscaled
    const int live = !cs.done && !cs.breakdown;
    s_live[tid] = live;
    if (live) {
      s_beta[tid] = cdiv(sh_rho[tid], cs.rho);
      s_alpha[tid] = cs.alpha;
      s_c[tid] = cs.c;
      s_zs[tid] = cs.zs;
      s_nrm[tid] = sqrt(sh_nu[tid]) / cs.bnorm;
    }
  }
  __syncthreads();

  // 2. per (active shift, column): pi recurrence, shift coefficients, convergence
  const int par = a.par;
  const int32_t* lcur = a.list + ((int64_t)par * gridDim.x + cb) * K;
  int32_t* lnext = a.list + ((int64_t)(par ^ 1) * gridDim.x + cb) * K;
  const int ncur = a.cnt[par * gridDim.x + cb];
  const bool live_c = s_live[c];
  const bool brk_c = a.cols[cb * B + c].breakdown;
  for (int e = ln; e < ncur; e += PTS) {
    const int k = lcur[e];
    const int64_t o = ((int64_t)cb * K + k) * B + c;
    ShiftState st = a.sh[o];
    ShiftCoef cf;
    cf.upd = 0;
    if (st.active && live_c) {
      const double2 sigma = csub(a.z[o], s_zs[c]);
      const double2 al = s_alpha[c], cn = s_c[c];
      const double2 t1 = cadd(mk(1.0 + cn.x, cn.y), cmul(al, sigma));
      const double2 pin = csub(cmul(t1, st.pi), cmul(cn, st.pi_prev));
      const double2 qq = cdiv(st.pi, pin);
      cf.a = cmul(qq, al);
      cf.b = cmul(cmul(qq, qq), s_beta[c]);
      cf.f = cdiv(mk(1.0, 0.0), pin);
      cf.upd = 1;
      st.pi_prev = st.pi;
      st.pi = pin;
      st.est = s_nrm[c] / cabsd(pin);
      if (!cfinite(pin) || !(cabs2(pin) > 0.0) || !isfinite(st.est) || !cfinite(cf.a) ||
          !cfinite(cf.b)) {
        st.active = 0;
        st.status = ST_BREAKDOWN;
        st.iters = n + 1;
        cf.upd = 0;
      } else if (st.est <= a.tol) {
        st.active = 0;
        st.status = ST_CONVERGED;
        st.iters = n + 1;
      }
      a.sh[o] = st;
    } else if (st.active && brk_c) {
      st.active = 0;
      st.status = ST_BREAKDOWN;
      st.iters = n;
      a.sh[o] = st;
    }
    a.coef[o] = cf;
  }
  __syncthreads();

  // 3. stable compaction of the shifts still active in any column of the block
  int base = 0;
  for (int e0 = 0; e0 < ncur; e0 += WG) {
    const int e = e0 + tid;
    int keep = 0, k = -1;
    if (e < ncur) {
      k = lcur[e];
      for (int cc = 0; cc < B; ++cc) keep |= a.sh[((int64_t)cb * K + k) * B + cc].active;
    }
    s_scan[tid] = keep;
    __syncthreads();
    for (int off = 1; off < WG; off <<= 1) {  // inclusive scan
      const int v = tid >= off ? s_scan[tid - off] : 0;
      __syncthreads();
      s_scan[tid] += v;
      __syncthreads();
    }
    if (keep) lnext[base + s_scan[tid] - 1] = k;
    if (tid == WG - 1) s_total = s_scan[tid];
    __syncthreads();
    base += s_total;
    __syncthreads();
  }
  const int nnext = base;

  // 4. per column: active count and argmin |pi_{n+1}| over its active shifts (ties: lowest k)
  {
    double best = INFINITY;
    int bestk = 0x7fffffff, cnt = 0;
    for (int e = ln; e < nnext; e += PTS) {
      const int k = lnext[e];
      const ShiftState& st = a.sh[((int64_t)cb * K + k) * B + c];
      if (st.active) {
        ++cnt;
        const double m = cabsd(st.pi);
        if (m < best || (m == best && k < bestk)) { best = m; bestk = k; }
      }
    }
    s_best[tid] = best;
    s_bestk[tid] = bestk;
    s_scan[tid] = cnt;
  }
  __syncthreads();
  for (int s = PTS / 2; s >= 1; s >>= 1) {
    if (ln < s) {
      const double b2 = s_best[tid + s * B];
      const int k2 = s_bestk[tid + s * B];
      if (b2 < s_best[tid] || (b2 == s_best[tid] && k2 < s_bestk[tid])) {
        s_best[tid] = b2;
        s_bestk[tid] = k2;
      }
      s_scan[tid] += s_scan[tid + s * B];
    }
    __syncthreads();
  }
  if (tid < B) {
    s_cnt_col[tid] = s_scan[tid];
    s_argmin[tid] = s_bestk[tid];
  }
  __syncthreads();

  // 5. seed switch (Eq. A13) and column bookkeeping; stored buffers are rescaled
  //    lazily through ColState::scale (true r = scale * stored r).
  const bool last = (int64_t)(n + 1) >= a.max_iter;
  if (tid < B) {
    ColState& cs = a.cols[cb * B + tid];
    int sw = -1;
    if (s_live[tid]) {
      double2 alpha = s_alpha[tid], beta = s_beta[tid];
      double2 rho_new = sh_rho[tid];
      const ShiftState& sst = a.sh[((int64_t)cb * K + cs.seed) * B + tid];
      const int ntot = s_cnt_col[tid];
      if (a.seed_switch && !sst.active && ntot > 0 && !last) sw = s_argmin[tid];
      if (sw >= 0) {
        const ShiftState& t = a.sh[((int64_t)cb * K + sw) * B + tid];
        const double2 fn = t.pi, fc = t.pi_prev;  // pi^{(s,s~)}_{n+1}, pi^{(s,s~)}_n
        const double2 qq = cdiv(fc, fn);
        alpha = cmul(qq, alpha);                   // alpha^{(s~)}_n
        beta = cmul(cmul(qq, qq), beta);           // beta^{(s~)}_n
        rho_new = cdiv(rho_new, cmul(fn, fn));     // (r~_{n+1}, r~_{n+1})
        cs.scale[a.buf_new] = cdiv(cs.scale[a.buf_new], fn);
        cs.scale[a.buf_new ^ 1] = cdiv(cs.scale[a.buf_new ^ 1], fc);
        cs.zs = a.z[((int64_t)cb * K + sw) * B + tid];
        cs.seed = sw;
        cs.nswitch += 1;
        s_fn[tid] = fn;
        s_fc[tid] = fc;
      }
      cs.rho = rho_new;
      cs.alpha_prev = alpha;
      cs.beta_prev = beta;
      cs.iters = n + 1;
      if (ntot == 0 || last) cs.done = 1;
    } else if (cs.breakdown) {
      cs.done = 1;
    }
    s_sw[tid] = sw;
  }
  __syncthreads();
  // rebase pi of the active shifts of switched columns; max-iteration cut-off
  for (int e = ln; e < nnext; e += PTS) {
    const int k = lnext[e];
    ShiftState& st = a.sh[((int64_t)cb * K + k) * B + c];
    if (!st.active) continue;
    if (last) {
      st.active = 0;
      st.status = ST_MAXITER;
      st.iters = n + 1;
    } else if (s_sw[c] >= 0) {
      st.pi = cdiv(st.pi, s_fn[c]);
      st.pi_prev = cdiv(st.pi_prev, s_fc[c]);
    }
  }
  __syncthreads();
  if (tid == 0) {
    int any = 0;
    for (int cc = 0; cc < B; ++cc) any |= !a.cols[cb * B + cc].done;
    a.blk_active[cb] = any;
    a.blk_iter[cb] = n + 1;
    a.k5cnt[cb] = ncur;
    a.cnt[(par ^ 1) * gridDim.x + cb] = any ? nnext : 0;
  }
}

// ------------------------------------------------------------------ shift vectors (Eqs. A11-A12)
//   x^(k) += alpha^(k)_n p^(k);   p^(k) = r_{n+1}[S] / pi_{n+1} + beta^(k)_n p^(k)
// grid: (ceil(nS*B/WG), ceil(K/KCH), nb); each thread owns one (row of S, column)
// and walks a chunk of the block's active shift list.
template <typename T, int B, int KCH>
__global__ __launch_bounds__(WG) void k_shift(const typename cplx_of<T>::type* __restrict__ rnew,
                                               int64_t N, const int32_t* __restrict__ srow,
                                               int nS, const int32_t* __restrict__ list,
                                               const int32_t* __restrict__ k5cnt, int K,
                                               const ShiftCoef* __restrict__ coef,
                                               double2* __restrict__ x,
                                               typename cplx_of<T>::type* __restrict__ p) {
  using cT = typename cplx_of<T>::type;
  const int cb = blockIdx.z;
  const int cnt = k5cnt[cb];
  const int e0 = blockIdx.y * KCH;
  if (e0 >= cnt) return;
  const int e1 = min(e0 + KCH, cnt);
  const int64_t gid = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (gid >= (int64_t)nS * B) return;
  const int i = (int)(gid / B), c = (int)(gid % B);
  const int64_t row = srow ? (int64_t)srow[i] : (int64_t)i;
  const double2 rv = to_d(rnew[((int64_t)cb * N + row) * B + c]);
  const int32_t* l = list + (int64_t)cb * K;
  for (int e = e0; e < e1; ++e) {
    const int k = l[e];
    const int64_t so = ((int64_t)cb * K + k) * B + c;
    const ShiftCoef cf = coef[so];
    if (!cf.upd) continue;
    const int64_t vo = (((int64_t)cb * K + k) * nS + i) * B + c;
    const double2 xv = x[vo];
    const double2 pv = to_d(p[vo]);
    x[vo] = cadd(xv, cmul(cf.a, pv));
    p[vo] = from_d<cT>(cadd(cmul(cf.f, rv), cmul(cf.b, pv)));
  }
}

// ------------------------------------------------------------------ initialisation
// Krylov buffers r_{-1} = r_0 = e_j (both buffers), for each block column.
template <typename T, int B>
__global__ void k_init_r(typename cplx_of<T>::type* r0, typename cplx_of<T>::type* r1, int64_t N,
                         const int32_t* __restrict__ rhs, int R, int nb) {
  using cT = typename cplx_of<T>::type;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)nb * N * B;
  if (gid >= tot) return;
  const int c = (int)(gid % B);
  const int64_t pnt = (gid / B) % N;
  const int cb = (int)(gid / (N * B));
  const int j = cb * B + c;
  cT v{0, 0};
  if (j < R && rhs[j] == pnt) v.x = 1;
  r0[gid] = v;
  r1[gid] = v;
}

// x^(k) = 0, p^(k) = e_j[S] for every shift
template <typename T, int B>
__global__ void k_init_xp(double2* x, typename cplx_of<T>::type* p, const int32_t* __restrict__ srow,
                          int nS, int K, int nb, const int32_t* __restrict__ rhs, int R) {
  using cT = typename cplx_of<T>::type;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)nb * K * nS * B;
  if (gid >= tot) return;
  const int c = (int)(gid % B);
  const int i = (int)((gid / B) % nS);
  const int cb = (int)(gid / ((int64_t)B * nS * K));
  const int j = cb * B + c;
  const int64_t row = srow ? (int64_t)srow[i] : (int64_t)i;
  cT v{0, 0};
  if (j < R && rhs[j] == row) v.x = 1;
  x[gid] = mk(0, 0);
  p[gid] = v;
}

template <int B>
__global__ void k_init_state(ColState* cols, ShiftState* sh, ShiftCoef* coef, double2* zcol,
                             const double2* __restrict__ z, int K, int nb, int R, int seed0,
                             int32_t* list, int32_t* cnt, int32_t* k5cnt, int32_t* blk_active,
                             int32_t* blk_iter) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)nb * K * B;
  if (gid < tot) {
    const int c = (int)(gid % B);
    const int k = (int)((gid / B) % K);
    const int cb = (int)(gid / ((int64_t)B * K));
    const int j = cb * B + c;
    ShiftState st;
    st.pi_prev = mk(1, 0);
    st.pi = mk(1, 0);
    st.est = 1.0;
    st.iters = 0;
    st.active = j < R;
    st.status = j < R ? ST_MAXITER : ST_UNUSED;
    st.pad_ = 0;
    sh[gid] = st;
    ShiftCoef cf{};
    cf.upd = 0;
    coef[gid] = cf;
    zcol[gid] = z[k];
    if (c == 0) {
      list[(int64_t)cb * K + k] = k;
      list[((int64_t)nb + cb) * K + k] = k;
    }
  }
  if (gid < (int64_t)nb * B) {
    const int j = (int)gid;
    ColState cs{};
    cs.rho = mk(1, 0);
    cs.alpha_prev = mk(1, 0);
    cs.beta_prev = mk(0, 0);
    cs.alpha = mk(0, 0);
    cs.c = mk(0, 0);
    cs.zs = z[seed0];
    cs.scale[0] = mk(1, 0);
    cs.scale[1] = mk(1, 0);
    cs.bnorm = 1.0;
    cs.seed = seed0;
    cs.done = j >= R;
    cols[j] = cs;
  }
  if (gid < nb) {
    const int cb = (int)gid;
    const int any = cb * B < R;
    cnt[cb] = any ? K : 0;
    cnt[nb + cb] = 0;
    k5cnt[cb] = 0;
    blk_active[cb] = any;
    blk_iter[cb] = 0;
  }
}

// G[k][j][i] = x[cb][k][i][c]  (j = cb*B + c), complex128 or complex64
template <int B, typename O>
__global__ void k_gather_out(const double2* __restrict__ x, O* __restrict__ out, int K, int R,
                             int nS) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)K * R * nS;
  if (gid >= tot) return;
  const int i = (int)(gid % nS);
  const int j = (int)((gid / nS) % R);
  const int k = (int)(gid / ((int64_t)nS * R));
  const int cb = j / B, c = j % B;
  const double2 v = x[(((int64_t)cb * K + k) * nS + i) * B + c];
  O o;
  o.x = v.x;
  o.y = v.y;
  out[gid] = o;
}

// one complex128 vector <-> column 0 of a block buffer (for scocg_apply_h)
template <typename T, int B>
__global__ void k_scatter_col0(const double2* __restrict__ x, typename cplx_of<T>::type* blk,
                               int64_t N) {
  using cT = typename cplx_of<T>::type;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= N * B) return;
  const int c = (int)(gid % B);
  const int64_t pnt = gid / B;
  cT v{0, 0};
  if (c == 0) v = from_d<cT>(x[pnt]);
  blk[gid] = v;
}

template <typename T, int B>
__global__ void k_gather_col0(const typename cplx_of<T>::type* __restrict__ blk, double2* y,
                              int64_t N) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= N) return;
  y[gid] = to_d(blk[gid * B]);
}

}  // namespace scocg
