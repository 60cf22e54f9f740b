// Device kernels of the shifted COCG solver (gfx950).
//
// Data layout in HBM (B = columns per block, 8 for complex128, 16 for complex64,
// so one grid point of one block is 128 contiguous bytes):
//   Krylov vectors      [nb][nz+2nf][nx*ny][B] complex<T> (RHS innermost; nf zero planes
//                       below and above the grid)
//   shift vectors x, p  [nb][K][nS][B]    x complex128, p complex<T>
//   shift state         [nb][K][B]        ShiftState (pi_{n-1}, pi_n, status)
//   column state        [nb*B]            ColState (seed scalars, FP64)
// Per seed iteration n the host enqueues three launches:
//   k_stencil<MU>     partials of mu_n = (r_n, A r_n),  A = z_s - H    (Eq. A5); in extra
//                     workgroups of the same launch: the projector contraction
//                     C_a = P_a^T r_n, the control step of iteration n-1 (control_body:
//                     beta (Eq. A6); pi, alpha^(i), beta^(i) per shift (Eqs. A8-A10);
//                     convergence, compaction of active shifts; seed switch (Eq. A13)),
//                     and the x^(i), p^(i) update of iteration n-2 on the rows S
//                     (Eqs. A11-A12 with Eq. A7)
//   k_alpha     alpha_n, c_n = beta_{n-1} alpha_n / alpha_{n-1}       (Eq. A5)
//   k_stencil<UPDATE> r_{n+1} = (1+c_n) r_n - alpha_n A r_n - c_n r_{n-1}  (Eq. A3), in place
//                     over r_{n-1}; partials of rho_{n+1}, ||r_{n+1}||^2
// and, at the end of each poll chunk, the control step of its last iteration alone
// (k_control, so that the host poll sees it); after the last iteration k_shift runs
// the two x, p updates still pending.  A r_n is recomputed in the UPDATE pass instead
// of being stored, so one iteration streams r_n twice, r_{n-1} once and writes r_{n+1}
// once.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

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

// Pointers held in argument tables (device memory, read by every workgroup of a
// batched launch) are typed global in device code, so the compiler emits global
// rather than flat memory instructions through them; the host sees plain pointers
// of the same size.
#if defined(__HIP_DEVICE_COMPILE__)
#define SCOCG_GLOBAL __attribute__((address_space(1)))
#else
#define SCOCG_GLOBAL
#endif
template <typename U>
using gptr = SCOCG_GLOBAL U*;
template <typename U>
__host__ __device__ inline gptr<U> to_g(U* p) {
  return (gptr<U>)p;
}

// ------------------------------------------------------------------ state records
struct ColState {
  double2 rho;         // (r_n, r_n) of the current seed (unscaled true value)
  double2 alpha_prev;  // alpha_{n-1}
  double2 beta_prev;   // beta_{n-1}
  double2 alpha;       // alpha_n (set by k_alpha)
  double2 c;           // beta_{n-1} alpha_n / alpha_{n-1}
  double2 zs;          // current seed energy
  double2 zs_mu;       // the seed energy the next mu pass uses (set by k_alpha; a seed
                       // switch in the control step running beside that pass changes zs
                       // only, and k_alpha corrects for the difference)
  double2 scale[2];    // stored Krylov buffer b holds r / scale[b] (lazy seed-switch rescale)
  double2 ar, ah, ap;  // r_{n+1} = ar r^st_n + ah (H r^st_n) + ap r^st_{n-1}
  double bnorm;        // ||b||
  double tol;          // per-column tolerance (0: the solve's tol)
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
  int32_t status;   // 0 converged, 1 max-iter, 2 breakdown, 3 unused column, 4 stalled
  int32_t active;   // still iterating
  int32_t best_it;  // iteration of the last halving of est (stagnation test)
  double best;      // est at that iteration
};

struct ShiftCoef {
  double2 a;   // alpha^(i)_n
  double2 b;   // beta^(i)_n
  double2 f;   // 1 / pi_{n+1} times the stored-buffer scale
  int32_t upd; // 1: apply this iteration
  int32_t pad_[3];
};

// Most list entries (energies) a shift workgroup takes; the LDS staging of their
// coefficients holds SHIFT_KCH_MAX x B records.
constexpr int SHIFT_KCH_MAX = 16;

enum { ST_CONVERGED = 0, ST_MAXITER = 1, ST_BREAKDOWN = 2, ST_UNUSED = 3, ST_STALLED = 4 };

// Real stencil coefficients, by value in the kernel argument segment.
template <typename T> struct Coefs {
  T cx[5], cy[5], cz[5];
  T c0;  // cx[0] + cy[0] + cz[0]
};

// ------------------------------------------------------------------ stencil pass
enum { MODE_MU = 0, MODE_UPDATE = 1, MODE_APPLY = 2 };

// launch geometry of a stencil pass: tile variant, tiles per plane, z-chunks,
// partial slots per column block, and the XCD-sliced 1-D grid
struct StencilGrid {
  int variant, ntx, nty, zc, nzc, nwg, nper, grid;
};

template <typename T>
struct ProjArgs {
  using cT = typename cplx_of<T>::type;
  gptr<const int32_t> aptr;   // [n_atoms+1] atom-major CSR
  gptr<const int32_t> aidx;   // [E] grid index
  gptr<const T> aval;         // [E][4]
  gptr<const T> aD;           // [n_atoms][4]
  int n_proj, n_atoms;
  gptr<cT> dc;                // out [nb][n_atoms][4][B]: D_l C_l
  gptr<double2> qa;           // out [nb][n_atoms][B]: sum_l C_l D_l C_l (null: not needed)
  int mfma;                   // complex64 columns: contract on FP32 matrix cores
};

template <typename T>
struct ShiftArgs {
  using cT = typename cplx_of<T>::type;
  gptr<const cT> rnew[2];          // plane 0 of the Krylov buffers; r_{n+1} is rnew[par ^ 1]
  int64_t bstride;            // elements per column block
  gptr<const int32_t> srow;        // [nS] rows S (null: all N rows)
  int nS;
  gptr<const int32_t> list;        // [3][nb][K] active shift lists (iteration m: m mod 3)
  gptr<const int32_t> k5cnt;       // [2][nb] entries of iteration m's update (m mod 2)
  int K, nb;
  gptr<const ShiftCoef> coef;      // [2][nb][K][B] by iteration parity
  gptr<double2> x;                 // [nb][K][nS][B]
  gptr<cT> p;                      // [nb][K][nS][B]
  int gx, gy;                 // workgroups per block along rows and along the list
  int kch;                    // list entries (energies) per workgroup
  int sym;                    // 1: S is the RHS set and block cb keeps rows i >= cb*B only
  int nt;                     // 1: x, p outgrow the last-level cache; stream them nontemporally
};

template <typename T>
struct StencilArgs {
  using cT = typename cplx_of<T>::type;
  gptr<const cT> r;           // [nb][nz+2NF][nxy][B] stored r_n, from the first padding plane
  gptr<cT> io;                // same layout; UPDATE: r_{n-1} in, r_{n+1} out; APPLY: H r out
  gptr<cT> bufs[2];           // pingpong: r = bufs[cur], io = bufs[cur ^ 1] (r, io unused)
  int pingpong;
  int64_t bstride;       // elements per column block ((nz+2NF)*nxy*B)
  gptr<const T> vloc;         // [N]
  Coefs<T> co;
  int nx, ny, nz, nxy;
  int ntx, nty;          // x-y tiles per plane
  int zc, nzc;           // planes per workgroup, z-chunks per plane column
  int nb;                // column blocks in the launch
  int nper;              // workgroups per XCD slice of the launch (grid = 8 * nper)
  gptr<const int32_t> prow;   // [N+1] point -> projector entries (null if no atoms)
  gptr<const int32_t> patom;  // [E] atom of each entry
  gptr<const T> pval;         // [E][4] projector values
  gptr<const cT> dc;          // [nb][n_atoms][4][B] D_a P_a^T r
  int n_atoms;
  gptr<const cT> pcv;         // [nb][n_ent][B] P_a D_a P_a^T r per atom-major entry (null:
                              // apply from dc inside the pass)
  gptr<const int32_t> pent;   // [E] atom-major entry of each point-major entry
  int n_ent;
  gptr<const ColState> cols;  // [nb*B]
  gptr<const int32_t> blk_active;  // [nb] (null: all active)
  gptr<double2> part0;        // [nb][nwg][B] mu or rho partials, nwg = nzc*ntx*nty
  gptr<double> part1;         // [nb][nwg][B] ||r||^2 partials (UPDATE)
  int nproj_wg;          // MU: leading workgroups doing the projector contraction
  ProjArgs<T> proj;
  int nshift_wg;         // MU: next workgroups doing the x, p update of iteration n - 2
  ShiftArgs<T> shift;
  int cache_mode;        // UPDATE: 0 r_{n-1} loads and r_{n+1} stores nontemporal; 1 r_{n+1}
                         // stores ordinary (the next mu pass reads them); 2 both ordinary
};

// Component-wise select of two complex values taken by value.  Register arrays
// of complex values must never meet a select of two aggregate lvalues: the
// compiler turns that into a select of addresses and moves the arrays to
// scratch memory.
template <typename V>
__device__ __forceinline__ V csel(bool c, V a, V b) {
  V r;
  r.x = c ? a.x : b.x;
  r.y = c ? a.y : b.y;
  return r;
}

// Streaming accesses that are not re-read by another workgroup (r_{n-1} in, r_{n+1}
// out): nontemporal, so they do not displace the r_n planes whose halos neighbouring
// workgroups still read from L2.
template <typename V>
__device__ __forceinline__ V ld_stream(const V* p) {
  using E = decltype(p->x);
  typedef E v2 __attribute__((ext_vector_type(2)));
  const v2 t = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
  V r;
  r.x = t.x;
  r.y = t.y;
  return r;
}
template <typename V>
__device__ __forceinline__ void st_stream(V* p, V v) {
  using E = decltype(v.x);
  typedef E v2 __attribute__((ext_vector_type(2)));
  v2 t;
  t.x = v.x;
  t.y = v.y;
  __builtin_nontemporal_store(t, reinterpret_cast<v2*>(p));
}

__device__ __forceinline__ int wrapi(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// Batched launches: workgroups [off[r], off[r+1]) of a launch serve region r
// (off[0] = 0, ascending, off[nreg] = grid).  Returns r for workgroup b.
__device__ __forceinline__ int region_of(const int32_t* __restrict__ off, int nreg, int b) {
  int lo = 0, hi = nreg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------------ projector contraction
// For one (atom a, column block): C_l = sum_e P_a[e][l] r[idx_e][c];  dc = D_l C_l;
// qa = sum_l C_l D_l C_l = r^T P_a D_a P_a^T r (the atom's share of r^T H r).
// Runs with NT threads; the reduction over entry lanes is a fixed tree in smem.
// r points at plane 0 of block 0; bstride = elements per column block.
template <typename T, int B, int NT>
__device__ __forceinline__ void proj_contract(const typename cplx_of<T>::type* __restrict__ r,
                                              int64_t bstride, const ProjArgs<T>& pa, int at,
                                              int cb, char* smem) {
  using cT = typename cplx_of<T>::type;
  constexpr int PL = NT / B;
  const int tid = threadIdx.x, c = tid % B, ln = tid / B;
  const cT* rb = r + (int64_t)cb * bstride + c;
  T acc[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  const int e0 = pa.aptr[at], e1 = pa.aptr[at + 1];
  for (int e = e0 + ln; e < e1; e += PL) {
    const cT v = rb[(int64_t)pa.aidx[e] * B];
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const T pv = pa.aval[(int64_t)e * 4 + l];
      acc[l][0] += pv * v.x;
      acc[l][1] += pv * v.y;
    }
  }
  T* sh = reinterpret_cast<T*>(smem);  // [4][2][NT]
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    sh[(l * 2 + 0) * NT + tid] = acc[l][0];
    sh[(l * 2 + 1) * NT + tid] = acc[l][1];
  }
  __syncthreads();
  for (int s = PL / 2; s >= 1; s >>= 1) {
    if (ln < s) {
#pragma unroll
      for (int q = 0; q < 8; ++q) sh[q * NT + tid] += sh[q * NT + tid + s * B];
    }
    __syncthreads();
  }
  if (ln == 0) {
    cT* o = pa.dc + ((int64_t)cb * pa.n_atoms + at) * 4 * B + c;
    double2 q = mk(0, 0);
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const T d = l < pa.n_proj ? pa.aD[at * 4 + l] : (T)0;
      const T cr = sh[(l * 2 + 0) * NT + tid], ci = sh[(l * 2 + 1) * NT + tid];
      cT v;
      v.x = d * cr;
      v.y = d * ci;
      o[l * B] = v;
      // C_l (D_l C_l), unconjugated
      q.x += (double)cr * v.x - (double)ci * v.y;
      q.y += (double)cr * v.y + (double)ci * v.x;
    }
    if (pa.qa) pa.qa[((int64_t)cb * pa.n_atoms + at) * B + c] = q;
  }
}

// The same contraction for complex64 columns (B = 16, i.e. 32 real columns) on FP32
// matrix cores.  v_mfma_f32_4x4x1_16b_f32 forms 16 independent 4x4 outer products per
// wave: block b (lanes 4b..4b+3, q = lane % 4) multiplies the 4 channels of one entry,
// A[q] = P[e][q], by 4 real columns of it, B[q] = X[e][4 (b % 8) + q], accumulating
// into D[i][q] (register i of lane 4b + q = channel i, column 4 (b % 8) + q).  Blocks
// 0-7 take entry e, blocks 8-15 entry e + 1, so one instruction covers two entries x 32
// columns with no padded rows.  Waves split the atom's entries; the two entry halves
// are added across lanes l and l + 32, then the waves in a fixed order through LDS.
typedef float scocg_v4f __attribute__((ext_vector_type(4)));

template <int NT>
__device__ __forceinline__ void proj_contract_mfma(const float2* __restrict__ r, int64_t bstride,
                                                   const ProjArgs<float>& pa, int at, int cb,
                                                   char* smem) {
  constexpr int B = 16, NW = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int blk = lane >> 2, q = lane & 3, half = blk >> 3, g = blk & 7;
  const float* rb = reinterpret_cast<const float*>(r + (int64_t)cb * bstride);
  const int e0 = pa.aptr[at], e1 = pa.aptr[at + 1];
  scocg_v4f acc = {0.f, 0.f, 0.f, 0.f};
  // U entry pairs per step: their gathers are all in flight before the first MFMA
  constexpr int U = 4;
  for (int eb = e0 + 2 * w; eb < e1; eb += 2 * NW * U) {
    float av[U], bv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = eb + 2 * NW * u + half;
      av[u] = 0.f;
      bv[u] = 0.f;
      if (e < e1) {
        av[u] = pa.aval[(int64_t)e * 4 + q];
        bv[u] = rb[(int64_t)pa.aidx[e] * (2 * B) + 4 * g + q];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc = __builtin_amdgcn_mfma_f32_4x4x1f32(av[u], bv[u], acc, 0, 0, 0);
  }
  // entry halves: lanes l and l + 32 hold the same (channel, column) set
  float v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = acc[i] + __shfl_xor(acc[i], 32);
  float* sh = reinterpret_cast<float*>(smem);  // [NW][4][32]
  if (lane < 32) {
#pragma unroll
    for (int i = 0; i < 4; ++i) sh[(w * 4 + i) * 32 + 4 * g + q] = v[i];
  }
  __syncthreads();
  float* cs = sh + NW * 4 * 32;  // [4][32]: C (channel, real column), waves summed in order
  if (tid < 128) {
    float t = 0.f;
    for (int ww = 0; ww < NW; ++ww) t += sh[ww * 128 + tid];
    cs[tid] = t;
  }
  __syncthreads();
  if (tid < B) {
    const int c = tid;
    float2* o = pa.dc + ((int64_t)cb * pa.n_atoms + at) * 4 * B + c;
    double2 qq = mk(0, 0);
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const float d = l < pa.n_proj ? pa.aD[at * 4 + l] : 0.f;
      const float cr = cs[l * 32 + 2 * c], ci = cs[l * 32 + 2 * c + 1];
      float2 vv;
      vv.x = d * cr;
      vv.y = d * ci;
      o[l * B] = vv;
      qq.x += (double)cr * vv.x - (double)ci * vv.y;
      qq.y += (double)cr * vv.y + (double)ci * vv.x;
    }
    if (pa.qa) pa.qa[((int64_t)cb * pa.n_atoms + at) * B + c] = qq;
  }
}

// The application P_a (D_a C_a) for complex64 columns on FP32 matrix cores, as
// per-entry products pc[cb][e][c] = sum_l P[e][l] (D_l C_l)[c] over the atom-major
// entries e of atom `at` (the operator pass then adds them at their points).
// v_mfma_f32_16x16x4f32 multiplies 16 entries x 4 channels (A: lane l holds
// P[e_0 + l % 16][l / 16]) by 4 channels x 16 real columns (B: lane l holds channel
// l / 16, real column l % 16 of D C), giving 16 entries x 16 columns (lane l: entries
// e_0 + 4 (l / 16) + v in register v, column l % 16); two instructions cover the 32
// real columns of a block.  Waves take 16-entry tiles in turn.
template <int NT>
__global__ __launch_bounds__(NT) void k_proj_apply_mfma(ProjArgs<float> pa, int n_ent,
                                                        float2* __restrict__ pc) {
  constexpr int B = 16, NW = NT / 64;
  const int at = blockIdx.x, cb = blockIdx.y;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const float2* dca = pa.dc + ((int64_t)cb * pa.n_atoms + at) * 4 * B;
  const float2 d0 = dca[kq * B + (col >> 1)], d1 = dca[kq * B + 8 + (col >> 1)];
  const float b0 = (col & 1) ? d0.y : d0.x, b1 = (col & 1) ? d1.y : d1.x;
  const int e0 = pa.aptr[at], e1 = pa.aptr[at + 1];
  float* out = reinterpret_cast<float*>(pc + (int64_t)cb * n_ent * B);
  for (int eb = e0 + 16 * w; eb < e1; eb += 16 * NW) {
    const int e = eb + col;
    const float av = e < e1 ? pa.aval[(int64_t)e * 4 + kq] : 0.f;
    const scocg_v4f z = {0.f, 0.f, 0.f, 0.f};
    const scocg_v4f r0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, b0, z, 0, 0, 0);
    const scocg_v4f r1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, b1, z, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = eb + 4 * kq + v;
      if (row < e1) {
        out[(int64_t)row * 2 * B + col] = r0[v];
        out[(int64_t)row * 2 * B + 16 + col] = r1[v];
      }
    }
  }
}

// the contraction on the path the handle chose (matrix cores for complex64 columns on
// request, else the vector ALUs)
template <typename T, int B, int NT>
__device__ __forceinline__ void proj_contract_any(const typename cplx_of<T>::type* __restrict__ r,
                                                  int64_t bstride, const ProjArgs<T>& pa, int at,
                                                  int cb, char* smem) {
  if constexpr (std::is_same<T, float>::value && B == 16) {
    if (pa.mfma) {
      proj_contract_mfma<NT>(r, bstride, pa, at, cb, smem);
      return;
    }
  }
  proj_contract<T, B, NT>(r, bstride, pa, at, cb, smem);
}

template <typename T, int B>
__global__ __launch_bounds__(WG) void k_proj(const typename cplx_of<T>::type* __restrict__ r,
                                              int64_t bstride, ProjArgs<T> pa,
                                              const int32_t* __restrict__ blk_active) {
  __shared__ __align__(16) char smem[8 * WG * sizeof(T)];
  const int at = blockIdx.x, cb = blockIdx.y;
  if (blk_active && !blk_active[cb]) return;
  proj_contract_any<T, B, WG>(r, bstride, pa, at, cb, smem);
}

// Stencil pass over one (x-y tile, z-chunk, column block).
//
// Krylov vectors are stored per column block as nz + 2*NF planes: NF zero
// planes below and above the transition region, so that the z-neighbours of
// every plane are plain loads (the truncation of the T block in z).  The
// workgroup stages plane iz of its TX x TY tile plus its halo in LDS (two
// buffers, alternating per plane, one barrier per plane) and keeps, per owned
// (point, column), the 2*NF+1 z-neighbours in a register queue that rotates
// instead of shifting: the z-march is unrolled by 2*NF+1 so that the queue slot
// of each plane is a compile-time index.  Loads for plane iz+1 (queue entry at
// iz+1+NF, halo ring, r_{n-1}) are issued before plane iz is computed.  Global
// addresses are a workgroup-uniform 64-bit base plus a 32-bit lane offset.
// Workgroup ids are remapped so that each XCD owns a contiguous run of
// (block, z-chunk, tile) indices: tiles that share halos share an L2.
//
// FULL: the tile lies inside the x-y plane (no ragged points).
//
// MODE_MU forms partials of r^T (z_s - H_loc) r = sum_p r_p ((z_s - d_p) r_p - 2 sum_{axis,
// k>0} c_k r_{p+k}) (H symmetric; every index pair (p, p+k) of the periodic or truncated
// axis is counted once), so it needs only the forward neighbours and a one-sided halo;
// the projector share r^T P D P^T r comes from the contraction (qa).  z_s is the seed
// energy k_alpha left for the pass (ColState::zs_mu): a control step running beside
// the pass may switch the seed, and k_alpha then adds (z_s,new - z_s,pass) (r, r).
template <typename T>
__device__ __forceinline__ T fmat(T a, T b, T c);
template <>
__device__ __forceinline__ double fmat<double>(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float fmat<float>(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}

template <typename T, int NF, int B, int MODE, int TX, int TY, int NT, bool FULL>
struct StencilWG {
  using cT = typename cplx_of<T>::type;
  // z-queue: logical index d holds plane iz - LO + d, d = 0 .. W-1.  The UPDATE and
  // APPLY passes need planes iz-NF .. iz+NF; the symmetric mu form only the centre
  // and its forward neighbours iz .. iz+NF, which halves its queue registers.
  static constexpr bool SYM = MODE == MODE_MU;
  static constexpr int LO = SYM ? 0 : NF;
  static constexpr int W = SYM ? NF + 1 : 2 * NF + 1;
  static constexpr int O = SYM ? 0 : NF;  // interior origin inside the LDS tile
  static constexpr int PX = TX + (SYM ? NF : 2 * NF);
  static constexpr int PY = TY + (SYM ? NF : 2 * NF);
  static constexpr int PL = NT / B;  // point lanes
  static_assert(NT % B == 0 && (TX * TY) % PL == 0, "tile must split evenly over point lanes");
  static constexpr int OPT = TX * TY / PL;  // owned points per thread per plane
  // halo ring of the cross-shaped stencil: the bands above and below the interior
  // rows over the interior columns only, then the side pieces of the interior rows
  // (the tile corners are never read, so they are never loaded)
  static constexpr int BAND = (PY - TY) * TX;
  static constexpr int RING = BAND + TY * (PX - TX);
  static constexpr int HPT = (RING + PL - 1) / PL;  // halo slots per thread
  static_assert(RING % 8 == 0, "idle halo slots must fill whole waves");
  // one spare slot per column absorbs the writes of unused halo lanes
  static constexpr int TILE_BYTES = (PX * PY + 1) * B * (int)sizeof(cT);
  static constexpr int RED_BYTES = NT * (int)(sizeof(double2) + sizeof(double));
  // after the two tile buffers: the UPDATE coefficients (ar, ah, ap) of the B columns
  static constexpr int COEF_OFF = 2 * TILE_BYTES;
  static constexpr int COEF_BYTES = 3 * B * (int)sizeof(double2);
  static constexpr int SMEM =
      COEF_OFF + COEF_BYTES > RED_BYTES ? COEF_OFF + COEF_BYTES : RED_BYTES;
  static constexpr uint32_t ESZ = sizeof(cT);

  const StencilArgs<T>& a;
  const cT* rsrc;  // r_n (padded, block 0)
  cT* iodst;       // UPDATE/APPLY output (padded, block 0)
  char* smem;
  int c, cb, z0, z1, nxy;
  int zmir;  // >= 0: this z-chunk marches downwards (physical plane = zmir - virtual)
  const char* rbase;  // uniform: this block's vector, first padding plane
  char* iobase;       // uniform: the UPDATE/APPLY output vector of this block
  uint32_t pstride;   // bytes per plane
  uint32_t qoff[OPT], hoff[HPT];  // lane byte offsets inside a plane
  int iofs[OPT], hl[HPT], gq[OPT];
  int nh;  // halo slots of this lane that hold ring points (the rest stay idle)
  bool val[OPT];
  cT Q[OPT][W];
  cT pq[OPT], ph[HPT], pp[OPT];
  T zr, zi;  // MU: the seed energy of the pass
  double2 acc0;
  double acc1;

  __device__ __forceinline__ StencilWG(const StencilArgs<T>& args, const cT* r, cT* io, char* sm)
      : a(args), rsrc(r), iodst(io), smem(sm) {}

  __device__ __forceinline__ const cT& ldr(uint32_t plane_pad, uint32_t lane_off) const {
    return *reinterpret_cast<const cT*>(rbase + plane_pad * pstride + lane_off);
  }

  // returns false if the workgroup has nothing to do
  __device__ __forceinline__ bool setup(int lid) {
    const int t = threadIdx.x, pl = t / B;
    c = t % B;
    const int ntile = a.ntx * a.nty;
    const int tile = lid % ntile;
    const int zci = (lid / ntile) % a.nzc;
    cb = lid / (ntile * a.nzc);
    if (a.blk_active && !a.blk_active[cb]) return false;
    const int x0 = (tile % a.ntx) * TX, y0 = (tile / a.ntx) * TY;
    z0 = zci * a.zc;
    z1 = min(z0 + a.zc, a.nz);
    nxy = a.nxy;
    const int nx = a.nx, ny = a.ny;
    pstride = (uint32_t)nxy * B * ESZ;
    rbase = reinterpret_cast<const char*>(rsrc + (int64_t)cb * a.bstride);
    iobase = (MODE == MODE_MU) ? nullptr : reinterpret_cast<char*>(iodst + (int64_t)cb * a.bstride);
#pragma unroll
    for (int m = 0; m < OPT; ++m) {
      const int pi = pl + m * PL;
      const int tx = pi % TX, ty = pi / TX;
      const int gx = x0 + tx, gy = y0 + ty;
      val[m] = FULL || (gx < nx && gy < ny);
      iofs[m] = ((ty + O) * PX + tx + O) * B + c;
      gq[m] = wrapi(gy, ny) * nx + wrapi(gx, nx);
      qoff[m] = ((uint32_t)gq[m] * B + c) * ESZ;
    }
    // halo slots h = pl + i * PL: the interior-width bands above and below the
    // interior rows, then the side pieces of the interior rows; slots past the ring
    // (i >= nh; whole waves, as RING is a multiple of the 8 point lanes of a wave)
    // neither load nor store
    nh = pl < RING ? (RING - 1 - pl) / PL + 1 : 0;
#pragma unroll
    for (int i = 0; i < HPT; ++i) {
      const int h = pl + i * PL;
      int sx = O, sy = 0;
      if (h < BAND) {
        const int rr = h / TX;
        sy = rr < O ? rr : rr + TY;
        sx = O + h % TX;
      } else if (h < RING) {
        const int q = h - BAND;
        sy = O + q / (PX - TX);
        const int s2 = q % (PX - TX);
        sx = s2 < O ? s2 : s2 + TX;
      }
      hl[i] = (h < RING ? sy * PX + sx : PX * PY) * B + c;
      const int g = wrapi(y0 + sy - O, ny) * nx + wrapi(x0 + sx - O, nx);
      hoff[i] = ((uint32_t)g * B + c) * ESZ;
    }
    if (MODE == MODE_UPDATE && pl == 0) {  // read after the first plane's barrier
      const ColState& cs = a.cols[cb * B + c];
      double2* sc = reinterpret_cast<double2*>(smem + COEF_OFF);
      sc[c] = cs.ar;
      sc[B + c] = cs.ah;
      sc[2 * B + c] = cs.ap;
    }
    if (MODE == MODE_MU) {
      const double2 zs = a.cols[cb * B + c].zs_mu;
      zr = (T)zs.x;
      zi = (T)zs.y;
    }
    acc0 = mk(0, 0);
    acc1 = 0.0;
    // odd z-chunks of the UPDATE/APPLY passes march downwards: the queue planes that
    // neighbouring chunks share are then read by both at about the same time (both
    // chunks start, or both end, at their common boundary), and the second read hits
    // L2.  The march runs over virtual planes z0..z1-1 either way; a downward chunk
    // maps virtual plane v to z0+z1-1-v (the operator is symmetric in z).  The
    // symmetric mu form counts forward pairs and keeps every chunk upwards.
    zmir = (!SYM && (zci & 1)) ? z0 + z1 - 1 : -1;
    // queue planes z0-LO .. z0-LO+W-2 into slots 0 .. W-2 (rotation 0); the first
    // step fills slot W-1; ragged points keep zeros
#pragma unroll
    for (int m = 0; m < OPT; ++m) {
#pragma unroll
      for (int d = 0; d < W - 1; ++d) {
        cT v = ldr((uint32_t)(pz(z0 - LO + d) + NF), qoff[m]);
        if (!FULL) {
          cT zero;
          zero.x = 0;
          zero.y = 0;
          v = csel(val[m], v, zero);
        }
        Q[m][d] = v;
      }
    }
    prefetch(z0);
    return true;
  }

  // physical plane of virtual plane v (uniform)
  __device__ __forceinline__ int pz(int v) const { return zmir >= 0 ? zmir - v : v; }

  // queue entry of virtual plane iz+NF for owned points (a ragged point instead
  // takes the wrapped value of plane iz, which only fills its LDS slot); r_{n-1} at
  // plane iz; halo ring of plane iz
  __device__ __forceinline__ void prefetch(int iz) {
    const uint32_t pc = (uint32_t)(pz(iz) + NF);  // padded physical index of plane iz
#pragma unroll
    for (int m = 0; m < OPT; ++m) {
      const uint32_t zq = (FULL || val[m]) ? (uint32_t)(pz(iz + NF) + NF) : pc;
      pq[m] = ldr(zq, qoff[m]);
      if (MODE == MODE_UPDATE)
        pp[m] = a.cache_mode < 2
                    ? ld_stream(reinterpret_cast<const cT*>(iobase + pc * pstride + qoff[m]))
                    : *reinterpret_cast<const cT*>(iobase + pc * pstride + qoff[m]);
    }
#pragma unroll
    for (int i = 0; i < HPT; ++i)
      if (i < nh) ph[i] = ldr(pc, hoff[i]);
  }

  // one (virtual) plane with queue rotation S: logical queue index d (plane
  // iz-LO+d) lives in slot (d + S) % W
  template <int S>
  __device__ __forceinline__ void step(int iz) {
    constexpr int snew = (W - 1 + S) % W;  // plane iz + NF, prefetched
    constexpr int sctr = (LO + S) % W;     // plane iz
    cT* lds = reinterpret_cast<cT*>(smem + ((iz - z0) & 1) * TILE_BYTES);
    // V and the projector range of this plane (the barrier covers part of their latency)
    const int ip = pz(iz);  // physical plane
    const T* vb = a.vloc + (int64_t)ip * nxy;
    T cv[OPT];
    int ce0[OPT], ce1[OPT];
    cT cp[OPT];
#pragma unroll
    for (int m = 0; m < OPT; ++m) {
      cv[m] = vb[gq[m]];
      if (MODE != MODE_MU) {
        ce0[m] = ce1[m] = 0;
        if (a.prow) {  // uniform branch
          const int32_t* pr = a.prow + (int64_t)ip * nxy + gq[m];
          ce0[m] = pr[0];
          ce1[m] = pr[1];
        }
      }
      if (FULL) {
        Q[m][snew] = pq[m];
        lds[iofs[m]] = Q[m][sctr];
      } else {
        cT zero;
        zero.x = 0;
        zero.y = 0;
        Q[m][snew] = csel(val[m], pq[m], zero);
        lds[iofs[m]] = csel(val[m], Q[m][sctr], pq[m]);
      }
      if (MODE == MODE_UPDATE) cp[m] = pp[m];
    }
#pragma unroll
    for (int i = 0; i < HPT; ++i)
      if (i < nh) lds[hl[i]] = ph[i];
    // readers of this buffer (plane iz-2) passed the previous plane's barrier
    // before these writes, so one barrier per plane suffices
    __syncthreads();
    if (iz + 1 < z1) prefetch(iz + 1);

#pragma unroll
    for (int m = 0; m < OPT; ++m) {
      if (!FULL && !val[m]) continue;
      const cT ctr = Q[m][sctr];
      const cT* L = lds + iofs[m];
      if constexpr (SYM) {
        // t = (z_s - d_p) r_p - 2 sum_k c_k (r_{p+k x} + r_{p+k y} + r_{p+k z});  mu += r_p t
        // (z_s - d_p formed per point: no cancellation between z_s (r, r) and r^T H r)
        T fr = 0, fi = 0;
#pragma unroll
        for (int k = 1; k <= NF; ++k) {
          const cT zp = Q[m][(LO + k + S) % W];
          fr = fmat(a.co.cz[k], zp.x, fr);
          fi = fmat(a.co.cz[k], zp.y, fi);
        }
        // x then y neighbours from LDS, fenced so that at most NF reads are in flight
        // (the 64-VGPR budget of two workgroups per CU)
#pragma unroll
        for (int k = 1; k <= NF; ++k) {
          const cT xp = L[k * B];
          fr = fmat(a.co.cx[k], xp.x, fr);
          fi = fmat(a.co.cx[k], xp.y, fi);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 1; k <= NF; ++k) {
          const cT yp = L[k * PX * B];
          fr = fmat(a.co.cy[k], yp.x, fr);
          fi = fmat(a.co.cy[k], yp.y, fi);
        }
        const T dr = zr - (a.co.c0 + cv[m]);
        const T tr = fmat(dr, ctr.x, fmat(-zi, ctr.y, (T)-2 * fr));
        const T ti = fmat(dr, ctr.y, fmat(zi, ctr.x, (T)-2 * fi));
        const double cr = ctr.x, ci = ctr.y;
        acc0.x = __builtin_fma(cr, (double)tr, __builtin_fma(-ci, (double)ti, acc0.x));
        acc0.y = __builtin_fma(cr, (double)ti, __builtin_fma(ci, (double)tr, acc0.y));
      } else {
        const T dg = a.co.c0 + cv[m];
        T hr = dg * ctr.x, hi = dg * ctr.y;
#pragma unroll
        for (int k = 1; k <= NF; ++k) {
          const cT zp = Q[m][(LO + k + S) % W], zm = Q[m][(LO - k + S) % W];
          hr = fmat(a.co.cz[k], zp.x + zm.x, hr);
          hi = fmat(a.co.cz[k], zp.y + zm.y, hi);
        }
        // x then y neighbours from LDS; the scheduling fence keeps the compiler
        // from hoisting all 4*NF reads at once (register pressure)
#pragma unroll
        for (int k = 1; k <= NF; ++k) {
          const cT xp = L[k * B], xm = L[-k * B];
          hr = fmat(a.co.cx[k], xp.x + xm.x, hr);
          hi = fmat(a.co.cx[k], xp.y + xm.y, hi);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 1; k <= NF; ++k) {
          const cT yp = L[k * PX * B], ym = L[-k * PX * B];
          hr = fmat(a.co.cy[k], yp.x + ym.x, hr);
          hi = fmat(a.co.cy[k], yp.y + ym.y, hi);
        }
        if (a.pcv) {  // uniform: the per-entry products were formed beforehand
          for (int e = ce0[m]; e < ce1[m]; ++e) {
            const cT v = a.pcv[((int64_t)cb * a.n_ent + a.pent[e]) * B + c];
            hr += v.x;
            hi += v.y;
          }
        } else {
          for (int e = ce0[m]; e < ce1[m]; ++e) {
            const cT* dca = a.dc + ((int64_t)cb * a.n_atoms + a.patom[e]) * 4 * B + c;
            const T* pvv = a.pval + (int64_t)e * 4;
#pragma unroll
            for (int l = 0; l < 4; ++l) {
              const cT d = dca[l * B];
              hr = fmat(pvv[l], d.x, hr);
              hi = fmat(pvv[l], d.y, hi);
            }
          }
        }
        cT* op = reinterpret_cast<cT*>(iobase + (uint32_t)(ip + NF) * pstride + qoff[m]);
        if (MODE == MODE_APPLY) {
          cT o;
          o.x = hr;
          o.y = hi;
          *op = o;
        } else {
          // r_{n+1} = ar r_n + ah (H r_n) + ap r_{n-1} (stored units; ar folds in z_s)
          const double2* sc = reinterpret_cast<const double2*>(smem + COEF_OFF);
          const double2 ar = sc[c], ah = sc[B + c], ap = sc[2 * B + c];
          const double2 rc = to_d(ctr), rp = to_d(cp[m]);
          const double hx = hr, hy = hi;
          double2 rn;
          rn.x = ar.x * rc.x;
          rn.x = __builtin_fma(-ar.y, rc.y, rn.x);
          rn.x = __builtin_fma(ah.x, hx, rn.x);
          rn.x = __builtin_fma(-ah.y, hy, rn.x);
          rn.x = __builtin_fma(ap.x, rp.x, rn.x);
          rn.x = __builtin_fma(-ap.y, rp.y, rn.x);
          rn.y = ar.x * rc.y;
          rn.y = __builtin_fma(ar.y, rc.x, rn.y);
          rn.y = __builtin_fma(ah.x, hy, rn.y);
          rn.y = __builtin_fma(ah.y, hx, rn.y);
          rn.y = __builtin_fma(ap.x, rp.y, rn.y);
          rn.y = __builtin_fma(ap.y, rp.x, rn.y);
          const cT rs = from_d<cT>(rn);
          if (a.cache_mode == 0)
            st_stream(op, rs);
          else
            *op = rs;
          const double2 rq = to_d(rs);
          acc0.x = __builtin_fma(rq.x, rq.x, __builtin_fma(-rq.y, rq.y, acc0.x));
          acc0.y = __builtin_fma(2.0 * rq.x, rq.y, acc0.y);
          acc1 = __builtin_fma(rq.x, rq.x, __builtin_fma(rq.y, rq.y, acc1));
        }
      }
    }
  }

  // up to W consecutive planes starting at rotation S
  template <int S>
  __device__ __forceinline__ void steps(int iz) {
    if constexpr (S < W) {
      if (iz < z1) {
        step<S>(iz);
        steps<S + 1>(iz + 1);
      }
    }
  }

  __device__ __forceinline__ void march() {
    for (int iz = z0; iz < z1; iz += W) steps<0>(iz);
  }

  // fixed-order workgroup reduction over the point lanes of each column
  __device__ __forceinline__ void reduce_and_store(int slot) {
    const int t = threadIdx.x, pl = t / B;
    __syncthreads();  // the tile buffers become reduction scratch
    double2* s0 = reinterpret_cast<double2*>(smem);
    double* s1 = reinterpret_cast<double*>(smem + NT * sizeof(double2));
    s0[t] = acc0;
    if (MODE == MODE_UPDATE) s1[t] = acc1;
    __syncthreads();
#pragma unroll
    for (int s = PL / 2; s >= 1; s >>= 1) {
      if (pl < s) {
        s0[t] = cadd(s0[t], s0[t + s * B]);
        if (MODE == MODE_UPDATE) s1[t] += s1[t + s * B];
      }
      __syncthreads();
    }
    if (pl == 0) {
      const int nwg = a.nzc * a.ntx * a.nty;
      const int64_t o = ((int64_t)cb * nwg + slot) * B + c;
      a.part0[o] = s0[t];
      if (MODE == MODE_UPDATE) a.part1[o] = s1[t];
    }
  }
};

// ------------------------------------------------------------------ column control
struct ControlArgs {
  gptr<const double2> part_rho;  // [nb][nwg][B]
  gptr<const double> part_nu;    // [nb][nwg][B]
  int nwg;
  gptr<ColState> cols;
  gptr<ShiftState> sh;           // [nb][K][B]
  gptr<ShiftCoef> coef;          // [2][nb][K][B] by iteration parity
  gptr<const double2> z;         // [nb][K][B] energies per column
  int K;
  gptr<int32_t> list;            // [3][nb][K] active shift lists, iteration n uses n mod 3
  gptr<int32_t> cnt;             // [3][nb] their lengths
  gptr<int32_t> k5cnt;           // [2][nb] list entries of iteration n's x, p update (n mod 2)
  gptr<double> pim;              // [nb][K][B] |pi_{n+1}| scratch (inside the mu launch)
  gptr<unsigned char> act;       // [nb][K][B] activity scratch (inside the mu launch)
  gptr<int32_t> blk_active;      // [nb]
  gptr<int32_t> blk_iter;        // [nb]
  int nb;                   // column blocks
  double tol;
  int64_t max_iter;
  int seed_switch;
  int stall;                // > 0 (complex64 recurrences): freeze a pair whose est is
                            // below 1e-2 and has not halved in max(stall, n/2) iterations
  double floor_est;         // complex64 recurrences: freeze at est <= max(tol, floor_est)
};

template <int B, int CTH>
struct CtlShared;
template <int B, int CTH>
__device__ __forceinline__ void control_body(const ControlArgs& a, int cb, int par, int lsel,
                                             CtlShared<B, CTH>& sm, double* pim,
                                             unsigned char* act);
template <typename T, int B, int NTH>
__device__ __forceinline__ void shift_body(const ShiftArgs<T>& a, int lb, int par, int lsel,
                                           char* smem);

// Stencil pass kernel.  MODE_MU launches additionally carry the projector
// contraction of r_n: the first nproj_wg workgroups (a multiple of 8, so the
// XCD slicing of the stencil workgroups is unchanged) each contract one
// (atom, column block).
// The mu pass fits two 1024-thread workgroups per CU (8 waves per SIMD, its short
// queue and one-sided halo keep it within 64 VGPRs and 62 KB of LDS); the others one.
template <typename T, int NF, int B, int MODE, int TX, int TY, int NT, bool FULL>
__global__ __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu(MODE == MODE_MU && NT == 1024 ? 8 : 4)))
void k_stencil(const StencilArgs<T>* __restrict__ regs, const int32_t* __restrict__ off,
               int nreg, int cur, const ControlArgs* __restrict__ cregs,
               const int32_t* __restrict__ coff, int nctl, int n6) {
  using SW = StencilWG<T, NF, B, MODE, TX, TY, NT, FULL>;
  using cT = typename cplx_of<T>::type;
  constexpr int PROJ_BYTES = 8 * NT * (int)sizeof(T);
  __shared__ __align__(16) char smem[SW::SMEM > PROJ_BYTES ? SW::SMEM : PROJ_BYTES];
  static_assert(PROJ_BYTES >= SHIFT_KCH_MAX * B * (int)sizeof(ShiftCoef),
                "the shift workgroups stage their coefficients in this buffer");
  static_assert(sizeof(CtlShared<B, NT>) <= sizeof(smem),
                "the control workgroups keep their reductions in this buffer");
  int bid = blockIdx.x;
  // MU launch of iteration n (n6 = n mod 6, cur = n mod 2): the first nctl workgroups
  // (every region's column blocks, table cregs / coff) run the control step of
  // iteration n - 1, which this pass does not depend on (its partials are independent
  // of the seed and of the lazy scales); its [K][B] scratch is global here
  if (MODE == MODE_MU && nctl > 0) {
    if (bid < nctl) {
      const int crg = region_of(coff, nreg, bid);
      const ControlArgs ca = cregs[crg];
      const int cb = bid - coff[crg];
      const int64_t o = (int64_t)cb * ca.K * B;
      control_body<B, NT>(ca, cb, cur ^ 1, (n6 + 5) % 3,
                          *reinterpret_cast<CtlShared<B, NT>*>(smem), ca.pim + o, ca.act + o);
      return;
    }
    bid -= nctl;
  }
  const int rg = region_of(off, nreg, bid);
  // a private copy: the compiler keeps the uniform fields in scalar registers instead
  // of reloading them from the table after every global store
  const StencilArgs<T> a = regs[rg];
  bid -= off[rg];
  // (selects, not a dynamic index: the copy of the table entry must stay in registers)
  const cT* rsrc = a.pingpong ? (cur ? a.bufs[1] : a.bufs[0]) : a.r;
  cT* iodst = a.pingpong ? (cur ? a.bufs[0] : a.bufs[1]) : a.io;
  if (MODE == MODE_MU && a.nproj_wg > 0) {
    if (bid < a.nproj_wg) {
      const int na = a.proj.n_atoms;
      if (bid >= na * a.nb) return;
      const int at = bid % na, cb = bid / na;
      if (a.blk_active && !a.blk_active[cb]) return;
      // plane-0 view of the padded vector
      proj_contract_any<T, B, NT>(rsrc + (int64_t)NF * a.nxy * B, a.bstride, a.proj, at, cb,
                                  smem);
      return;
    }
    bid -= a.nproj_wg;
  }
  if (MODE == MODE_MU && a.nshift_wg > 0) {
    // the x, p update of iteration n - 2 (parity cur, list (n - 2) mod 3, coefficients
    // from the control step of n - 2, which finished in the previous launch): it reads
    // r_{n-1}[S], which stays in the other buffer until this iteration's r_{n+1} pass,
    // and x, p, which no other workgroup touches
    if (bid < a.nshift_wg) {
      if (bid < a.shift.gx * a.shift.gy * a.shift.nb)
        shift_body<T, B, NT>(a.shift, bid, cur, (n6 + 4) % 3, smem);
      return;
    }
    bid -= a.nshift_wg;
  }
  // XCD-aware decode of the logical stencil workgroup id
  const int ntile = a.ntx * a.nty;
  const int total = a.nb * a.nzc * ntile;
  const int lid = (bid % 8) * a.nper + bid / 8;
  if (lid >= total) return;
  SW w(a, rsrc, iodst, smem);
  if (!w.setup(lid)) return;
  w.march();
  if (MODE == MODE_APPLY) return;
  w.reduce_and_store(lid % (a.nzc * ntile));
}

// ------------------------------------------------------------------ seed alpha (Eq. A5)
// One workgroup per column block: fixed-order reduction of the mu partials, then
//   alpha_n = rho_n / (mu_n - beta_{n-1}/alpha_{n-1} rho_n),  c_n = beta_{n-1} alpha_n / alpha_{n-1}
// and the coefficients of the UPDATE pass in stored-buffer units.
struct AlphaArgs {
  gptr<const double2> part;        // [nb][nwg][B] mu partials
  int nwg;
  gptr<const double2> qa;          // [nb][n_atoms][B] projector shares
  int n_atoms;
  gptr<ColState> cols;             // [nb*B]
  gptr<const int32_t> blk_active;  // [nb]
};

// one workgroup per column block of every region (off: blocks per region)
template <int B>
__global__ __launch_bounds__(WG) void k_alpha(const AlphaArgs* __restrict__ regs,
                                               const int32_t* __restrict__ off, int nreg,
                                               int buf_cur) {
  constexpr int PTS = WG / B;
  const int rg = region_of(off, nreg, blockIdx.x);
  const AlphaArgs ar = regs[rg];
  const auto part = ar.part;
  const auto qa = ar.qa;
  const int nwg = ar.nwg, n_atoms = ar.n_atoms;
  const auto cols = ar.cols;
  const auto blk_active = ar.blk_active;
  const int tid = threadIdx.x, c = tid % B, ln = tid / B, cb = blockIdx.x - off[rg];
  if (!blk_active[cb]) return;
  // (r^st)^T (z_pass - H) r^st = sum of the local stencil partials - sum over atoms of
  // r^T P D P^T r, z_pass = cs.zs_mu
  double2 acc = mk(0, 0);
  for (int w = ln; w < nwg; w += PTS) acc = cadd(acc, part[((int64_t)cb * nwg + w) * B + c]);
  for (int at = ln; at < n_atoms; at += PTS) acc = csub(acc, qa[((int64_t)cb * n_atoms + at) * B + c]);
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
    cs.ar = cs.ah = cs.ap = mk(0, 0);
    return;
  }
  const double2 s_cur = cs.scale[buf_cur], s_prev = cs.scale[buf_cur ^ 1];
  // stored r^st = r / s  =>  mu = r^T (z_s - H) r = s^2 (r^st)^T (z_pass - H) r^st
  // + (z_s - z_pass) (r, r) (unconjugated bilinear forms; cs.rho holds the true (r, r);
  // the second term is zero unless the seed switched in the control step beside the pass)
  const double2 mu = cadd(cmul(cmul(s_cur, s_cur), sh[tid]),
                          cmul(csub(cs.zs, cs.zs_mu), cs.rho));
  cs.zs_mu = cs.zs;  // for the next mu pass
  const double2 denom = csub(mu, cmul(cdiv(cs.beta_prev, cs.alpha_prev), cs.rho));
  const double2 alpha = cdiv(cs.rho, denom);
  const double2 cc = cdiv(cmul(cs.beta_prev, alpha), cs.alpha_prev);
  if (!(cabs2(denom) > 0.0) || !(cabs2(cs.rho) > 0.0) || !cfinite(alpha) || !cfinite(cc)) {
    cs.breakdown = 1;
    cs.ar = cs.ah = cs.ap = mk(0, 0);
    return;
  }
  cs.alpha = alpha;
  cs.c = cc;
  // r_{n+1} = (1 + c_n) r_n - alpha_n (z_s - H) r_n - c_n r_{n-1}
  //         = (1 + c_n - alpha_n z_s) r_n + alpha_n H r_n - c_n r_{n-1}
  cs.ar = cmul(csub(mk(1.0 + cc.x, cc.y), cmul(alpha, cs.zs)), s_cur);
  cs.ah = cmul(alpha, s_cur);
  cs.ap = cmul(mk(-cc.x, -cc.y), s_prev);
}


// One workgroup per column block (B columns x K shifts):
//   beta_n = rho_{n+1} / rho_n                                            (Eq. A6)
//   pi_{n+1} = (1 + c_n + alpha_n sigma) pi_n - c_n pi_{n-1}, sigma = z_k - z_s   (Eq. A8)
//   alpha^(k)_n = pi_n/pi_{n+1} alpha_n,  beta^(k)_n = (pi_n/pi_{n+1})^2 beta_n  (Eqs. A9-A10)
//   freeze (k, j) once ||r_{n+1}|| / |pi_{n+1}| <= tol ||b|| (or, for complex64
//   vectors, once that estimate stops halving); compact the active list;
//   seed switch to the active shift of smallest |pi_{n+1}| once the seed froze (Eq. A13).
// Thread t always serves column t % B (CT is a multiple of B), so every
// per-column reduction is one fixed-order tree over the CT/B lanes of that
// column.  Activity flags and |pi_{n+1}| of the block live in dynamic LDS
// ([K][B] each) between the phases; the compaction uses wave ballots.
constexpr int CT = 1024;  // threads of the control kernel

// the reduction and per-column arrays of one control workgroup of CTH threads
template <int B, int CTH>
struct CtlShared {
  double2 sh_rho[CTH];
  double sh_nu[CTH];
  int s_k[CTH];
  double2 s_alpha[B], s_beta[B], s_c[B], s_zs[B], s_fn[B], s_fc[B], s_rhon[B];
  double s_nrm[B], s_tol[B];
  int s_live[B], s_sw[B];
  int s_wsum[CTH / 64];
  int s_any_sw;
};

// One column block's control step of iteration n: par = n mod 2 selects the Krylov
// buffers and the halves of the coefficients and update counts, lsel = n mod 3 the
// active list it reads (it writes list (n + 1) mod 3).  pim, act: [K][B] scratch of
// this block (LDS in k_control, global inside the mu launch).  Every thread of the
// workgroup calls it (it holds barriers).
template <int B, int CTH>
__device__ __forceinline__ void control_body(const ControlArgs& a, int cb, int par, int lsel,
                                             CtlShared<B, CTH>& sm, double* pim,
                                             unsigned char* act) {
  constexpr int PL = CTH / B;
  constexpr int NWAVE = CTH / 64;
  const int buf_new = par ^ 1;  // Krylov buffer holding r_{n+1}
  const int tid = threadIdx.x, c = tid % B, ln = tid / B;
  const int nb = a.nb;
  const int lnx = lsel == 2 ? 0 : lsel + 1;  // the list of iteration n + 1
  if (!a.blk_active[cb]) {
    if (tid == 0) a.k5cnt[par * nb + cb] = 0;
    return;
  }
  const int K = a.K;
  const int n = a.blk_iter[cb];
  double2* sh_rho = sm.sh_rho;
  double* sh_nu = sm.sh_nu;
  int* s_k = sm.s_k;
  double2 *s_alpha = sm.s_alpha, *s_beta = sm.s_beta, *s_c = sm.s_c, *s_zs = sm.s_zs,
          *s_fn = sm.s_fn, *s_fc = sm.s_fc, *s_rhon = sm.s_rhon;
  double *s_nrm = sm.s_nrm, *s_tol = sm.s_tol;
  int *s_live = sm.s_live, *s_sw = sm.s_sw, *s_wsum = sm.s_wsum;
  int& s_any_sw = sm.s_any_sw;

  // 1. reduce rho_{n+1} and ||r_{n+1}||^2 partials
  {
    double2 ra = mk(0, 0);
    double na = 0.0;
    for (int w = ln; w < a.nwg; w += PL) {
      const int64_t o = ((int64_t)cb * a.nwg + w) * B + c;
      ra = cadd(ra, a.part_rho[o]);
      na += a.part_nu[o];
    }
    sh_rho[tid] = ra;
    sh_nu[tid] = na;
  }
  __syncthreads();
  for (int s = PL / 2; s >= 1; s >>= 1) {
    if (ln < s) {
      sh_rho[tid] = cadd(sh_rho[tid], sh_rho[tid + s * B]);
      sh_nu[tid] += sh_nu[tid + s * B];
    }
    __syncthreads();
  }
  if (tid < B) {
    ColState& cs = a.cols[cb * B + tid];
    cs.scale[buf_new] = mk(1.0, 0.0);  // r_{n+1} was just written unscaled
    const int live = !cs.done && !cs.breakdown;
    s_live[tid] = live;
    s_rhon[tid] = sh_rho[tid];
    if (live) {
      s_beta[tid] = cdiv(sh_rho[tid], cs.rho);
      s_alpha[tid] = cs.alpha;
      s_c[tid] = cs.c;
      s_zs[tid] = cs.zs;
      s_nrm[tid] = sqrt(sh_nu[tid]) / cs.bnorm;
      s_tol[tid] = cs.tol > 0.0 ? cs.tol : a.tol;
    }
    if (tid == 0) s_any_sw = 0;
  }
  __syncthreads();

  // 2. per (active shift, column): pi recurrence, shift coefficients, convergence
  const int32_t* lcur = a.list + ((int64_t)lsel * nb + cb) * K;
  int32_t* lnext = a.list + ((int64_t)lnx * nb + cb) * K;
  const int ncur = a.cnt[lsel * nb + cb];
  const bool live_c = s_live[c];
  const bool brk_c = a.cols[cb * B + c].breakdown;
  for (int e = ln; e < ncur; e += PL) {
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
      } else if (st.est <= s_tol[c]) {
        st.active = 0;
        st.status = ST_CONVERGED;
        st.iters = n + 1;
      } else if (a.stall > 0) {
        // complex64 recurrences level off near u32 times the condition number: stop
        // at the floor, or once the estimate stalls past the initial plateau, and
        // leave the pair to the FP64-checked refinement
        if (st.est <= a.floor_est) {
          st.active = 0;
          st.status = ST_STALLED;
          st.iters = n + 1;
        } else if (st.est <= 0.5 * st.best) {
          st.best = st.est;
          st.best_it = n + 1;
        } else if (st.est < 1e-2 && n + 1 - st.best_it > max(a.stall, (n + 1) / 2)) {
          st.active = 0;
          st.status = ST_STALLED;
          st.iters = n + 1;
        }
      }
      a.sh[o] = st;
    } else if (st.active && brk_c) {
      st.active = 0;
      st.status = ST_BREAKDOWN;
      st.iters = n;
      a.sh[o] = st;
    }
    a.coef[(int64_t)par * nb * K * B + o] = cf;
    act[k * B + c] = (unsigned char)st.active;
    pim[k * B + c] = cabsd(st.pi);
  }
  __syncthreads();

  // 3. stable compaction of the shifts still active in any column of the block:
  //    rank inside each wave by ballot, wave offsets by a serial prefix over waves
  const int lane = tid & 63, wave = tid >> 6;
  int base = 0;
  for (int e0 = 0; e0 < ncur; e0 += CTH) {
    const int e = e0 + tid;
    int keep = 0, k = -1;
    if (e < ncur) {
      k = lcur[e];
#pragma unroll
      for (int cc = 0; cc < B; ++cc) keep |= act[k * B + cc];
    }
    const unsigned long long m = __ballot(keep);
    const int rank = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) s_wsum[wave] = __popcll(m);
    __syncthreads();
    int off = base;
    for (int w = 0; w < wave; ++w) off += s_wsum[w];
    if (keep) lnext[off + rank] = k;
    int tot = 0;
    for (int w = 0; w < NWAVE; ++w) tot += s_wsum[w];
    base += tot;
    __syncthreads();
  }
  const int nnext = base;

  // 4. per column: active count and argmin |pi_{n+1}| over its active shifts (ties: lowest k)
  {
    double best = INFINITY;
    int bestk = 0x7fffffff, cnt = 0;
    for (int e = ln; e < nnext; e += PL) {
      const int k = lnext[e];
      if (act[k * B + c]) {
        ++cnt;
        const double mm = pim[k * B + c];
        if (mm < best || (mm == best && k < bestk)) { best = mm; bestk = k; }
      }
    }
    sh_nu[tid] = best;
    s_k[tid] = bestk;
    sh_rho[tid].x = cnt;
  }
  __syncthreads();
  for (int s = PL / 2; s >= 1; s >>= 1) {
    if (ln < s) {
      const double b2 = sh_nu[tid + s * B];
      const int k2 = s_k[tid + s * B];
      if (b2 < sh_nu[tid] || (b2 == sh_nu[tid] && k2 < s_k[tid])) {
        sh_nu[tid] = b2;
        s_k[tid] = k2;
      }
      sh_rho[tid].x += sh_rho[tid + s * B].x;
    }
    __syncthreads();
  }
  int cnt_c = 0, argmin_c = 0;
  double pimin_c = INFINITY;
  if (tid < B) {
    cnt_c = (int)sh_rho[tid].x;
    argmin_c = s_k[tid];
    pimin_c = sh_nu[tid];
  }
  __syncthreads();  // sh_rho is reused below

  // 5. seed switch (Eq. A13) and column bookkeeping; stored buffers are rescaled
  //    lazily through ColState::scale (true r = scale * stored r).
  const bool last = (int64_t)(n + 1) >= a.max_iter;
  if (tid < B) {
    ColState& cs = a.cols[cb * B + tid];
    int sw = -1;
    if (s_live[tid]) {
      double2 alpha = s_alpha[tid], beta = s_beta[tid];
      double2 rho_new = s_rhon[tid];
      const ShiftState& sst = a.sh[((int64_t)cb * K + cs.seed) * B + tid];
      // complex64 vectors also switch while the seed is active, as soon as another
      // shift's residual is 4x the seed's (|pi| < 1/4; the seed's own pi is 1): the
      // seed then never sinks towards the rounding floor of its stored vectors, which
      // a later rebase by 1/pi would amplify
      const bool early = a.stall > 0 && sst.active && pimin_c < 0.25;
      if (a.seed_switch && (!sst.active || early) && cnt_c > 0 && !last) sw = argmin_c;
      if (sw >= 0) {
        const ShiftState& t = a.sh[((int64_t)cb * K + sw) * B + tid];
        const double2 fn = t.pi, fc = t.pi_prev;  // pi^{(s,s~)}_{n+1}, pi^{(s,s~)}_n
        const double2 qq = cdiv(fc, fn);
        alpha = cmul(qq, alpha);                   // alpha^{(s~)}_n
        beta = cmul(cmul(qq, qq), beta);           // beta^{(s~)}_n
        rho_new = cdiv(rho_new, cmul(fn, fn));     // (r~_{n+1}, r~_{n+1})
        cs.scale[buf_new] = cdiv(cs.scale[buf_new], fn);
        cs.scale[buf_new ^ 1] = cdiv(cs.scale[buf_new ^ 1], fc);
        cs.zs = a.z[((int64_t)cb * K + sw) * B + tid];
        cs.seed = sw;
        cs.nswitch += 1;
        s_fn[tid] = fn;
        s_fc[tid] = fc;
        s_any_sw = 1;
      }
      cs.rho = rho_new;
      cs.alpha_prev = alpha;
      cs.beta_prev = beta;
      cs.iters = n + 1;
      if (cnt_c == 0 || last) cs.done = 1;
    } else if (cs.breakdown) {
      cs.done = 1;
    }
    s_sw[tid] = sw;
  }
  __syncthreads();
  // rebase pi of the active shifts of switched columns; max-iteration cut-off
  if (s_any_sw || last) {
    for (int e = ln; e < nnext; e += PL) {
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
  }
  __syncthreads();
  if (tid == 0) {
    int any = 0;
    for (int cc = 0; cc < B; ++cc) any |= !a.cols[cb * B + cc].done;
    a.blk_active[cb] = any;
    a.blk_iter[cb] = n + 1;
    a.k5cnt[par * nb + cb] = ncur;
    a.cnt[lnx * nb + cb] = any ? nnext : 0;
  }
}

template <int B>
__global__ __launch_bounds__(CT) void k_control(const ControlArgs* __restrict__ regs,
                                                 const int32_t* __restrict__ off, int nreg,
                                                 int par, int lsel) {
  const int rg = region_of(off, nreg, blockIdx.x);
  const ControlArgs a = regs[rg];
  __shared__ CtlShared<B, CT> sm;
  extern __shared__ __align__(16) char dyn[];
  double* pim = reinterpret_cast<double*>(dyn);  // [K][B] |pi_{n+1}|
  unsigned char* act = reinterpret_cast<unsigned char*>(dyn + (size_t)a.K * B * sizeof(double));
  control_body<B, CT>(a, blockIdx.x - off[rg], par, lsel, sm, pim, act);
}

// ------------------------------------------------------------------ shift vectors (Eqs. A11-A12)
//   x^(k) += alpha^(k)_n p^(k);   p^(k) = r_{n+1}[S] / pi_{n+1} + beta^(k)_n p^(k)
// grid: (ceil(nS*B/WG), ceil(K/KCH), nb); each thread owns one (row of S, column)
// and walks a chunk of the block's active shift list.

// One (energy, row, column) update with its coefficients; explicit FMAs, so that every
// instance (and full and projected storage) rounds alike.
template <bool NT, typename cT>
__device__ __forceinline__ void shift_one(double2* __restrict__ x, cT* __restrict__ p, int64_t vo,
                                          const ShiftCoef& cf, double2 xv, double2 pv,
                                          double2 rv) {
  double2 xn, t, pn;
  xn.x = __builtin_fma(cf.a.x, pv.x, __builtin_fma(-cf.a.y, pv.y, xv.x));
  xn.y = __builtin_fma(cf.a.x, pv.y, __builtin_fma(cf.a.y, pv.x, xv.y));
  t.x = __builtin_fma(cf.b.x, pv.x, -(cf.b.y * pv.y));
  t.y = __builtin_fma(cf.b.x, pv.y, cf.b.y * pv.x);
  pn.x = __builtin_fma(cf.f.x, rv.x, __builtin_fma(-cf.f.y, rv.y, t.x));
  pn.y = __builtin_fma(cf.f.x, rv.y, __builtin_fma(cf.f.y, rv.x, t.y));
  if (NT) {
    st_stream(x + vo, xn);
    st_stream(p + vo, from_d<cT>(pn));
  } else {
    x[vo] = xn;
    p[vo] = from_d<cT>(pn);
  }
}

// The energy loop of one thread (row i of S, column c): x, p updates of the list
// entries e0..e1-1, two entries at a time so that four loads are in flight.  sc holds
// the coefficients of the entries, [e - e0][B], staged in LDS by the workgroup.
// NT: nontemporal x, p (they do not fit the last-level cache).
template <bool NT, int B, typename T>
__device__ __forceinline__ void shift_loop(const ShiftArgs<T>& a, const int32_t* l,
                                           const ShiftCoef* sc, int e0, int e1, int cb, int i,
                                           int c, double2 rv) {
  using cT = typename cplx_of<T>::type;
  double2* __restrict__ x = a.x;
  cT* __restrict__ p = a.p;
  const int64_t kstride = (int64_t)a.nS * B, rc = (int64_t)i * B + c, kb = (int64_t)cb * a.K;
  int e = e0;
  for (; e + 1 < e1; e += 2) {
    const ShiftCoef* s0 = sc + (e - e0) * B + c;
    const ShiftCoef* s1 = s0 + B;
    const int u0 = s0->upd, u1 = s1->upd;
    const int64_t v0 = (kb + l[e]) * kstride + rc, v1 = (kb + l[e + 1]) * kstride + rc;
    double2 x0 = mk(0, 0), x1 = mk(0, 0), p0 = mk(0, 0), p1 = mk(0, 0);
    if (u0) {
      x0 = NT ? ld_stream(x + v0) : x[v0];
      p0 = to_d(NT ? ld_stream(p + v0) : p[v0]);
    }
    if (u1) {
      x1 = NT ? ld_stream(x + v1) : x[v1];
      p1 = to_d(NT ? ld_stream(p + v1) : p[v1]);
    }
    if (u0) shift_one<NT>(x, p, v0, *s0, x0, p0, rv);
    if (u1) shift_one<NT>(x, p, v1, *s1, x1, p1, rv);
  }
  if (e < e1) {
    const ShiftCoef* s0 = sc + (e - e0) * B + c;
    if (s0->upd) {
      const int64_t v0 = (kb + l[e]) * kstride + rc;
      const double2 x0 = NT ? ld_stream(x + v0) : x[v0];
      const double2 p0 = to_d(NT ? ld_stream(p + v0) : p[v0]);
      shift_one<NT>(x, p, v0, *s0, x0, p0, rv);
    }
  }
}

// x^(k) += alpha^(k) p^(k);  p^(k) = r_{n+1}[S] / pi^(k)_{n+1} + beta^(k) p^(k)  (Eqs. A11-A12)
// for workgroup lb of one region (NTH threads): gx * gy * nb workgroups, NTH rows of S
// x kch list entries x column block.  The update of iteration m: par = m mod 2 (its
// Krylov buffer parity and the halves of its coefficients and counts), lsel = m mod 3
// (its active list).  smem: at least SHIFT_KCH_MAX * B * sizeof(ShiftCoef) bytes;
// every thread of the workgroup must call this (it holds a barrier).
template <typename T, int B, int NTH>
__device__ __forceinline__ void shift_body(const ShiftArgs<T>& a, int lb, int par, int lsel,
                                           char* smem) {
  using cT = typename cplx_of<T>::type;
  const int bx = lb % a.gx, by = (lb / a.gx) % a.gy, cb = lb / (a.gx * a.gy);
  const int cnt = a.k5cnt[par * a.nb + cb];
  const int e0 = by * a.kch;
  if (e0 >= cnt) return;  // uniform
  const int e1 = min(e0 + a.kch, cnt);
  const int K = a.K;
  const int32_t* l = a.list + ((int64_t)lsel * a.nb + cb) * K;
  // the chunk's coefficients are the same for every row: stage them once
  ShiftCoef* sc = reinterpret_cast<ShiftCoef*>(smem);
  const ShiftCoef* cf = a.coef + (int64_t)par * a.nb * K * B;
  for (int t = threadIdx.x; t < (e1 - e0) * B; t += NTH)
    sc[t] = cf[((int64_t)cb * K + l[e0 + t / B]) * B + t % B];
  __syncthreads();
  const int64_t gid = (int64_t)bx * NTH + threadIdx.x;
  if (gid >= (int64_t)a.nS * B) return;
  const int i = (int)(gid / B), c = (int)(gid % B);
  // complex symmetry: rows below the block's first column are the mirror of columns
  // already kept by an earlier block, G(S_i, e_j) = G(S_j, e_i)
  if (a.sym && i < cb * B) return;
  const int64_t row = a.srow ? (int64_t)a.srow[i] : (int64_t)i;
  const cT* rnew = par ? a.rnew[0] : a.rnew[1];  // r_{n+1}: buffer par ^ 1
  const double2 rv = to_d(rnew[(int64_t)cb * a.bstride + row * B + c]);
  if (a.nt)
    shift_loop<true, B, T>(a, l, sc, e0, e1, cb, i, c, rv);
  else
    shift_loop<false, B, T>(a, l, sc, e0, e1, cb, i, c, rv);
}

// Stand-alone x, p update of the last iteration of a solve (every other iteration's
// update runs in the next mu launch, overlapped with its stencil workgroups).
template <typename T, int B>
__global__ __launch_bounds__(WG) void k_shift(const ShiftArgs<T>* __restrict__ regs,
                                               const int32_t* __restrict__ off, int nreg,
                                               int par, int lsel) {
  __shared__ __align__(16) char smem[SHIFT_KCH_MAX * B * sizeof(ShiftCoef)];
  const int rg = region_of(off, nreg, blockIdx.x);
  const ShiftArgs<T> a = regs[rg];
  shift_body<T, B, WG>(a, blockIdx.x - off[rg], par, lsel, smem);
}

// ------------------------------------------------------------------ initialisation
// Krylov buffers r_{-1} = r_0 = e_j (both buffers, padding planes zero), for each
// block column; bstride = elements per block, pad = points before plane 0.
template <typename T, int B>
__global__ void k_init_r(typename cplx_of<T>::type* r0, typename cplx_of<T>::type* r1,
                         int64_t bstride, int64_t N, int64_t pad, const int32_t* __restrict__ rhs,
                         int R, int nb) {
  using cT = typename cplx_of<T>::type;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)nb * bstride;
  if (gid >= tot) return;
  const int cb = (int)(gid / bstride);
  const int64_t w = gid % bstride;
  const int c = (int)(w % B);
  const int64_t pnt = w / B - pad;
  const int j = cb * B + c;
  cT v{0, 0};
  if (j < R && pnt >= 0 && pnt < N && rhs[j] == pnt) v.x = 1;
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

// z: [K] energies shared by every column, or (zpc != null, K == 1) one energy per
// column zpc[cb*B + c]; tolc (optional, [R]): per-column tolerances.
template <int B>
__global__ void k_init_state(ColState* cols, ShiftState* sh, ShiftCoef* coef, double2* zcol,
                             const double2* __restrict__ z, const double2* __restrict__ zpc,
                             const double* __restrict__ tolc,
                             int K, int nb, int R, int seed0, int32_t* list, int32_t* cnt,
                             int32_t* k5cnt, int32_t* blk_active, int32_t* blk_iter) {
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
    st.best_it = 0;
    st.best = 1.0;
    sh[gid] = st;
    ShiftCoef cf{};
    cf.upd = 0;
    coef[gid] = cf;        // both parity halves
    coef[tot + gid] = cf;
    zcol[gid] = zpc ? zpc[cb * B + c] : z[k];
    if (c == 0) list[(int64_t)cb * K + k] = k;  // the list of iteration 0
  }
  if (gid < (int64_t)nb * B) {
    const int j = (int)gid;
    ColState cs{};
    cs.rho = mk(1, 0);
    cs.alpha_prev = mk(1, 0);
    cs.beta_prev = mk(0, 0);
    cs.alpha = mk(0, 0);
    cs.c = mk(0, 0);
    cs.zs = zpc ? zpc[j] : z[seed0];
    cs.zs_mu = cs.zs;
    cs.scale[0] = mk(1, 0);
    cs.scale[1] = mk(1, 0);
    cs.bnorm = 1.0;
    cs.tol = (tolc && j < R) ? tolc[j] : 0.0;
    cs.seed = seed0;
    cs.done = j >= R;
    cols[j] = cs;
  }
  if (gid < nb) {
    const int cb = (int)gid;
    const int any = cb * B < R;
    cnt[cb] = any ? K : 0;
    cnt[nb + cb] = 0;
    cnt[2 * nb + cb] = 0;
    k5cnt[cb] = 0;  // no x, p update is pending for iterations -2 and -1
    k5cnt[nb + cb] = 0;
    blk_active[cb] = any;
    blk_iter[cb] = 0;
  }
}

// ------------------------------------------------------------------ FP64 true residual
// t = b - (z - H) x in FP64 for x in the full-storage layout [nblk][N][B] (nblk =
// nb*K; block kb = cb*K + k holds x^(k) of columns cb*B..cb*B+B-1); b = e_j for a
// unit right-hand side (rhs != null) or a dense vector brhs [nblk][N][B] (null:
// zero).  One thread per (point, column), neighbours straight from memory (a
// one-off pass, not part of the iteration).  part[kb][wg][c] = sum |t|^2 over the
// workgroup's points; t is stored if tout != null.
template <int NF, int B>
__global__ __launch_bounds__(WG) void k_true_resid(
    const double2* __restrict__ x, double2* __restrict__ tout, const double* __restrict__ vloc,
    Coefs<double> co, int nx, int ny, int nz, const int32_t* __restrict__ prow,
    const int32_t* __restrict__ patom, const double* __restrict__ pval,
    const double2* __restrict__ dc, int n_atoms, const double2* __restrict__ zcol,
    const int32_t* __restrict__ rhs, int R, int K, double* __restrict__ part) {
  constexpr int PTS = WG / B;
  const int tid = threadIdx.x, c = tid % B, ln = tid / B;
  const int kb = blockIdx.y;
  const int cb = kb / K;
  const int nxy = nx * ny;
  const int64_t N = (int64_t)nxy * nz;
  const int64_t p = (int64_t)blockIdx.x * PTS + ln;
  double acc = 0.0;
  if (p < N) {
    const double2* xb = x + (int64_t)kb * N * B + c;
    const int ix = (int)(p % nx), iy = (int)((p / nx) % ny), iz = (int)(p / nxy);
    const double2 xc = xb[p * B];
    const double dg = co.c0 + vloc[p];
    double hr = dg * xc.x, hi = dg * xc.y;
    for (int k = 1; k <= NF; ++k) {
      const int64_t xp = (int64_t)iz * nxy + iy * nx + wrapi(ix + k, nx);
      const int64_t xm = (int64_t)iz * nxy + iy * nx + wrapi(ix - k, nx);
      const int64_t yp = (int64_t)iz * nxy + wrapi(iy + k, ny) * nx + ix;
      const int64_t ym = (int64_t)iz * nxy + wrapi(iy - k, ny) * nx + ix;
      const double2 vxp = xb[xp * B], vxm = xb[xm * B], vyp = xb[yp * B], vym = xb[ym * B];
      hr += co.cx[k] * (vxp.x + vxm.x) + co.cy[k] * (vyp.x + vym.x);
      hi += co.cx[k] * (vxp.y + vxm.y) + co.cy[k] * (vyp.y + vym.y);
      if (iz + k < nz) {
        const double2 v = xb[(p + (int64_t)k * nxy) * B];
        hr += co.cz[k] * v.x;
        hi += co.cz[k] * v.y;
      }
      if (iz - k >= 0) {
        const double2 v = xb[(p - (int64_t)k * nxy) * B];
        hr += co.cz[k] * v.x;
        hi += co.cz[k] * v.y;
      }
    }
    if (prow) {
      for (int e = prow[p]; e < prow[p + 1]; ++e) {
        const double2* d = dc + ((int64_t)kb * n_atoms + patom[e]) * 4 * B + c;
        for (int l = 0; l < 4; ++l) {
          hr += pval[(int64_t)e * 4 + l] * d[l * B].x;
          hi += pval[(int64_t)e * 4 + l] * d[l * B].y;
        }
      }
    }
    const double2 z = zcol[(int64_t)kb * B + c];
    // t = b - z x + H x
    double2 t = mk(hr - (z.x * xc.x - z.y * xc.y), hi - (z.x * xc.y + z.y * xc.x));
    const int j = cb * B + c;
    if (rhs && j < R && rhs[j] == p) t.x += 1.0;
    if (tout) tout[(int64_t)kb * N * B + p * B + c] = t;
    acc = t.x * t.x + t.y * t.y;
  }
  __shared__ double sh[WG];
  sh[tid] = acc;
  __syncthreads();
  for (int s = PTS / 2; s >= 1; s >>= 1) {
    if (ln < s) sh[tid] += sh[tid + s * B];
    __syncthreads();
  }
  if (ln == 0) part[((int64_t)kb * gridDim.x + blockIdx.x) * B + c] = sh[tid];
}

// norm[kb*B + c] = sqrt(sum over the nwg partials), fixed order
template <int B>
__global__ __launch_bounds__(WG) void k_norms(const double* __restrict__ part, int nwg,
                                               double* __restrict__ norm) {
  constexpr int PTS = WG / B;
  const int tid = threadIdx.x, c = tid % B, ln = tid / B, kb = blockIdx.x;
  double acc = 0.0;
  for (int w = ln; w < nwg; w += PTS) acc += part[((int64_t)kb * nwg + w) * B + c];
  __shared__ double sh[WG];
  sh[tid] = acc;
  __syncthreads();
  for (int s = PTS / 2; s >= 1; s >>= 1) {
    if (ln < s) sh[tid] += sh[tid + s * B];
    __syncthreads();
  }
  if (ln == 0) norm[(int64_t)kb * B + c] = sqrt(sh[tid]);
}

// ------------------------------------------------------------------ dense right-hand sides
// r_{-1} = r_0 = b for dense right-hand sides (the refinement solves): column j
// of block cb (j = cb*B + c) takes src[src_kb[j]][pnt][src_c[j]] * scale[j] from a
// full-storage array of column width BS; padding planes and unused columns are
// zero.  grid (ceil(bstride / WG), nb); partials of b^T b and ||b||^2 of the
// stored (rounded) values per (block, workgroup, column).
template <typename T, int B, int BS>
__global__ __launch_bounds__(WG) void k_init_r_dense(
    typename cplx_of<T>::type* r0, typename cplx_of<T>::type* r1, int64_t bstride, int64_t N,
    int64_t pad, const double2* __restrict__ src, const int32_t* __restrict__ src_kb,
    const int32_t* __restrict__ src_c, const double* __restrict__ scale, int R,
    double2* __restrict__ prho, double* __restrict__ pnu) {
  using cT = typename cplx_of<T>::type;
  constexpr int PTS = WG / B;
  const int tid = threadIdx.x, c = tid % B, ln = tid / B;
  const int cb = blockIdx.y;
  const int64_t w = (int64_t)blockIdx.x * WG + tid;
  const int j = cb * B + c;
  cT v{0, 0};
  if (w < bstride) {
    const int64_t pnt = w / B - pad;
    if (j < R && pnt >= 0 && pnt < N) {
      const double2 s = src[((int64_t)src_kb[j] * N + pnt) * BS + src_c[j]];
      v = from_d<cT>(mk(s.x * scale[j], s.y * scale[j]));
    }
    r0[(int64_t)cb * bstride + w] = v;
    r1[(int64_t)cb * bstride + w] = v;
  }
  const double2 vd = to_d(v);
  __shared__ double2 s0[WG];
  __shared__ double s1[WG];
  s0[tid] = mk(vd.x * vd.x - vd.y * vd.y, 2.0 * vd.x * vd.y);
  s1[tid] = vd.x * vd.x + vd.y * vd.y;
  __syncthreads();
  for (int s = PTS / 2; s >= 1; s >>= 1) {
    if (ln < s) {
      s0[tid] = cadd(s0[tid], s0[tid + s * B]);
      s1[tid] += s1[tid + s * B];
    }
    __syncthreads();
  }
  if (ln == 0) {
    const int64_t o = ((int64_t)cb * gridDim.x + blockIdx.x) * B + c;
    prho[o] = s0[tid];
    pnu[o] = s1[tid];
  }
}

// rho_0 = b^T b and ||b|| of every column from the partials of k_init_r_dense
template <int B>
__global__ __launch_bounds__(WG) void k_dense_cols(const double2* __restrict__ prho,
                                                    const double* __restrict__ pnu, int nwg,
                                                    ColState* cols, int R) {
  constexpr int PTS = WG / B;
  const int tid = threadIdx.x, c = tid % B, ln = tid / B, cb = blockIdx.x;
  double2 a = mk(0, 0);
  double n = 0.0;
  for (int w = ln; w < nwg; w += PTS) {
    a = cadd(a, prho[((int64_t)cb * nwg + w) * B + c]);
    n += pnu[((int64_t)cb * nwg + w) * B + c];
  }
  __shared__ double2 s0[WG];
  __shared__ double s1[WG];
  s0[tid] = a;
  s1[tid] = n;
  __syncthreads();
  for (int s = PTS / 2; s >= 1; s >>= 1) {
    if (ln < s) {
      s0[tid] = cadd(s0[tid], s0[tid + s * B]);
      s1[tid] += s1[tid + s * B];
    }
    __syncthreads();
  }
  if (ln == 0 && cb * B + c < R) {
    ColState& cs = cols[cb * B + c];
    cs.rho = s0[tid];
    cs.bnorm = sqrt(s1[tid]);
  }
}

// full storage with K = 1: x = 0, p = b (the plane-0 view of the padded r_0)
template <typename T, int B>
__global__ void k_init_xp_dense(double2* x, typename cplx_of<T>::type* p,
                                const typename cplx_of<T>::type* __restrict__ r0p,
                                int64_t bstride, int64_t N, int nb) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)nb * N * B) return;
  const int cb = (int)(gid / (N * B));
  const int64_t w = gid % (N * B);
  x[gid] = mk(0, 0);
  p[gid] = r0p[(int64_t)cb * bstride + w];
}

// refinement update: x_out[src_kb[j]][pnt][src_c[j]] += back[j] * d[cb][pnt][c]
// (d: full-storage K = 1 solution, j = cb*B + c)
template <int B, int BS>
__global__ void k_add_correction(double2* __restrict__ xout, const double2* __restrict__ d,
                                 const int32_t* __restrict__ src_kb,
                                 const int32_t* __restrict__ src_c,
                                 const double* __restrict__ back,
                                 const ShiftState* __restrict__ inner, int R, int64_t N) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)R * N) return;
  const int j = (int)(gid / N);
  // a correction whose inner solve did not at least halve its residual is dropped
  if (!(inner[j].est < 0.5)) return;
  const int64_t pnt = gid % N;
  const int cb = j / B, c = j % B;
  const double2 dv = d[((int64_t)cb * N + pnt) * B + c];
  double2& xo = xout[((int64_t)src_kb[j] * N + pnt) * BS + src_c[j]];
  xo = mk(xo.x + back[j] * dv.x, xo.y + back[j] * dv.y);
}

// G[k][j][i] = x[cb][k][i][c]  (j = cb*B + c), complex128 or complex64.  sym: rows
// i < cb*B were not kept for block cb; they are row j of column i (S = RHS set).
template <int B, typename O>
__global__ void k_gather_out(const double2* __restrict__ x, O* __restrict__ out, int K, int R,
                             int nS, int sym) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)K * R * nS;
  if (gid >= tot) return;
  int i = (int)(gid % nS);
  int j = (int)((gid / nS) % R);
  const int k = (int)(gid / ((int64_t)nS * R));
  if (sym && i < (j / B) * B) {
    const int t = i;
    i = j;
    j = t;
  }
  const int cb = j / B, c = j % B;
  const double2 v = x[(((int64_t)cb * K + k) * nS + i) * B + c];
  O o;
  o.x = v.x;
  o.y = v.y;
  out[gid] = o;
}

// one complex128 vector <-> column 0 of a padded one-block buffer (for scocg_apply_h)
template <typename T, int B>
__global__ void k_scatter_col0(const double2* __restrict__ x, typename cplx_of<T>::type* blk,
                               int64_t bstride, int64_t N, int64_t pad) {
  using cT = typename cplx_of<T>::type;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= bstride) return;
  const int c = (int)(gid % B);
  const int64_t pnt = gid / B - pad;
  cT v{0, 0};
  if (c == 0 && pnt >= 0 && pnt < N) v = from_d<cT>(x[pnt]);
  blk[gid] = v;
}

template <typename T, int B>
__global__ void k_gather_col0(const typename cplx_of<T>::type* __restrict__ blk, double2* y,
                              int64_t N, int64_t pad) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= N) return;
  y[gid] = to_d(blk[(gid + pad) * B]);
}

}  // namespace scocg
