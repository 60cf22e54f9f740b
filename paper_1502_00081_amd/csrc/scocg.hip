// Host driver and C ABI of the shifted COCG Green's-function solver (see include/scocg.h).
//
// scocg_create uploads H once: the local potential, the stencil coefficients
// (kernel arguments) and the projector blocks in two CSR forms (by atom for the
// contraction C_a = P_a^T r, by grid point for the application P_a D_a C_a).
// scocg_solve plans the column blocks, initialises the seed and shift states
// on the device and runs the per-iteration kernel sequence of kernels.hpp until
// every (shift, column) pair has frozen, polling one flag array per
// `poll_every` iterations; the polled iterations can be replayed as one
// captured hipGraph.
#include <fcntl.h>
#include <hip/hip_runtime.h>
#include <unistd.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "kernels.hpp"
#include "obm_kernels.hpp"
#include "scocg.h"

using namespace scocg;

// Device workspace of the allocation-free entry point scocg_apply_h_noalloc: one copy
// per GPU, held from the library's first use on that GPU until the process ends.  In
// host code `scratch` names a host-side stand-in, not device memory: its address on
// each device is taken once with hipGetSymbolAddress (init_scratch, called by
// scocg_create with the handle's device current) and only that address is used.
static __device__ __align__(256) char scratch[SCOCG_SCRATCH_BYTES];

namespace {

thread_local std::string g_err;

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void hip_check(hipError_t e, const char* what, int line) {
  if (e == hipSuccess) return;
  const int code = (e == hipErrorOutOfMemory) ? SCOCG_ENOMEM : SCOCG_EHIP;
  throw Error(code, std::string(what) + " failed (line " + std::to_string(line) +
                        "): " + hipGetErrorString(e));
}
#define HIPCHK(x) hip_check((x), #x, __LINE__)
#define KCHK() hip_check(hipGetLastError(), "kernel launch", __LINE__)

void require(bool ok, const std::string& msg) {
  if (!ok) throw Error(SCOCG_EINVAL, msg);
}

// Owning device allocation.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void alloc(size_t n) {
    release();
    if (n == 0) return;
    HIPCHK(hipMalloc(&p, n));
    bytes = n;
  }
  template <typename U> U* as() const { return static_cast<U*>(p); }
};

// A HIP event that is destroyed on every path out of its scope (errors throw).
struct Event {
  hipEvent_t e = nullptr;
  Event() { HIPCHK(hipEventCreate(&e)); }
  Event(const Event&) = delete;
  Event& operator=(const Event&) = delete;
  Event(Event&& o) noexcept : e(o.e) { o.e = nullptr; }
  ~Event() {
    if (e) (void)hipEventDestroy(e);
  }
  operator hipEvent_t() const { return e; }
};

// device ms between two events recorded on a stream (waits for the second)
float elapsed_ms(const Event& a, const Event& b) {
  HIPCHK(hipEventSynchronize(b));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, a, b));
  return ms;
}

// A captured graph and its executable, destroyed on every path out of scope.
struct Graph {
  hipGraph_t g = nullptr;
  hipGraphExec_t x = nullptr;
  Graph() = default;
  Graph(const Graph&) = delete;
  Graph& operator=(const Graph&) = delete;
  ~Graph() {
    if (x) (void)hipGraphExecDestroy(x);
    if (g) (void)hipGraphDestroy(g);
  }
};

template <typename U>
void upload(DevBuf& b, const std::vector<U>& v, hipStream_t s) {
  b.alloc(v.size() * sizeof(U));
  if (!v.empty()) {
    HIPCHK(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(U), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  }
}

unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// SCOCG_TRACE=1 prints per-pass refinement statistics to stderr
// SCOCG_TRACE=1: solve summaries on stderr; 2: also a progress line every 2048 seed
// iterations (long solves)
int trace_level() {
  static const int lv = [] {
    const char* e = getenv("SCOCG_TRACE");
    return e ? atoi(e) : 0;
  }();
  return lv;
}
bool trace_on() { return trace_level() > 0; }

// device -> address of `scratch` on that device
std::mutex g_scratch_mu;
std::map<int, char*> g_scratch;

// once per device, with that device current
void init_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch.count(device)) return;
  void* p = nullptr;
  HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw Error(SCOCG_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
  g_scratch[device] = static_cast<char*>(p);
}

char* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch.find(device);
  if (it == g_scratch.end())
    throw Error(SCOCG_EHIP, "scratch of device " + std::to_string(device) + " not set up");
  return it->second;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
struct scocg_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;  // created here because the caller passed NULL
  int precision = SCOCG_FP64;
  int nx = 0, ny = 0, nz = 0, nxy = 0, nf = 4, n_proj = 0;
  int64_t N = 0;
  int n_atoms = 0;
  int proj_mfma = 0;  // complex64 columns: projector contraction on FP32 matrix cores
  std::string arch;   // device architecture (gcnArchName up to the first ':')
  std::vector<double> coef;  // [3][nf+1]
  // operator arrays on the device (T = double or float by precision)
  DevBuf vloc, aptr, aidx, aval, aD, prow, patom, pval, pent;
  int64_t n_ent = 0;  // projector entries (sum over atoms)
  // FP64 copies for the true-residual pass (aliases of the above for SCOCG_FP64)
  DevBuf vloc64, aval64, aD64, pval64;
  // last solve
  struct Solve {
    bool ok = false;
    int B = 0, nb = 0, K = 0, R = 0, nS = 0, nwg = 0;
    int Kout = 0;  // energies returned: K, or K - 1 when the last one is an auxiliary seed
    int sym = 0;   // rows below each block's first column are taken from the mirror column
    StencilGrid g{};
    int kch = 4;  // energies per workgroup of k_shift
    int cache_mode = 0;  // cache policy of the r_{n+1} pass (StencilArgs::cache_mode)
    int zc_mu = 0;       // z planes per workgroup of the mu pass (0: the same as g.zc)
    bool full = false;
    DevBuf r0, r1, z, cols, sh, coef, list, cnt, k5cnt, blk_active, blk_iter, rhs, srow, x, p,
        dc, qa, part0, part1, partm, pim, act;
    int32_t* h_flags = nullptr;
    ~Solve() {
      if (h_flags) (void)hipHostFree(h_flags);
    }
  };
  std::unique_ptr<Solve> last;
  // autotuned launch shapes per (B, column blocks, energies, rows): {tile, zchunk, kch}
  // {tile, zchunk, shift chunk, cache mode, mu-pass zchunk (0: the same as zchunk)}
  std::map<std::array<int64_t, 4>, std::array<int32_t, 5>> tuned;
};

namespace {

template <typename T>
Coefs<T> make_coefs(const scocg_ctx& h) {
  Coefs<T> co{};
  const int nf = h.nf;
  for (int k = 0; k <= nf; ++k) {
    co.cx[k] = (T)h.coef[0 * (nf + 1) + k];
    co.cy[k] = (T)h.coef[1 * (nf + 1) + k];
    co.cz[k] = (T)h.coef[2 * (nf + 1) + k];
  }
  co.c0 = (T)(h.coef[0] + h.coef[nf + 1] + h.coef[2 * (nf + 1)]);
  return co;
}

template <typename T>
void upload_operator(scocg_ctx& h, const double* vloc, const int64_t* atom_ptr,
                     const int64_t* atom_idx, const double* atom_P, const double* atom_D) {
  hipStream_t s = h.stream;
  std::vector<T> v(h.N);
  for (int64_t i = 0; i < h.N; ++i) v[i] = (T)vloc[i];
  upload(h.vloc, v, s);
  if (h.n_atoms == 0) return;
  const int np = h.n_proj;
  const int64_t E = atom_ptr[h.n_atoms];
  std::vector<int32_t> ap(h.n_atoms + 1), ai(E);
  std::vector<T> av(E * 4, (T)0), ad(h.n_atoms * 4, (T)0);
  for (int a = 0; a <= h.n_atoms; ++a) ap[a] = (int32_t)atom_ptr[a];
  for (int64_t e = 0; e < E; ++e) {
    ai[e] = (int32_t)atom_idx[e];
    for (int l = 0; l < np; ++l) av[e * 4 + l] = (T)atom_P[e * np + l];
  }
  for (int a = 0; a < h.n_atoms; ++a)
    for (int l = 0; l < np; ++l) ad[a * 4 + l] = (T)atom_D[a * np + l];
  // transpose to point-major CSR: entries of one point in atom order
  std::vector<int32_t> pr(h.N + 1, 0), pa(E), pe(E);
  std::vector<T> pv(E * 4);
  for (int64_t e = 0; e < E; ++e) pr[ai[e] + 1]++;
  for (int64_t i = 0; i < h.N; ++i) pr[i + 1] += pr[i];
  std::vector<int32_t> fill(pr.begin(), pr.end() - 1);
  for (int a = 0; a < h.n_atoms; ++a)
    for (int64_t e = ap[a]; e < ap[a + 1]; ++e) {
      const int32_t slot = fill[ai[e]]++;
      pa[slot] = a;
      pe[slot] = (int32_t)e;
      for (int l = 0; l < 4; ++l) pv[(int64_t)slot * 4 + l] = av[e * 4 + l];
    }
  h.n_ent = E;
  upload(h.pent, pe, s);
  upload(h.aptr, ap, s);
  upload(h.aidx, ai, s);
  upload(h.aval, av, s);
  upload(h.aD, ad, s);
  upload(h.prow, pr, s);
  upload(h.patom, pa, s);
  upload(h.pval, pv, s);
}

// FP64 operator data for the true-residual pass of a complex64 handle
void upload_operator64(scocg_ctx& h, const double* vloc, const int64_t* atom_ptr,
                       const int64_t* atom_idx, const double* atom_P, const double* atom_D) {
  hipStream_t s = h.stream;
  upload(h.vloc64, std::vector<double>(vloc, vloc + h.N), s);
  if (h.n_atoms == 0) return;
  const int np = h.n_proj;
  const int64_t E = atom_ptr[h.n_atoms];
  std::vector<double> av(E * 4, 0.0), ad(h.n_atoms * 4, 0.0), pv(E * 4, 0.0);
  std::vector<int32_t> pr(h.N + 1, 0);
  for (int64_t e = 0; e < E; ++e)
    for (int l = 0; l < np; ++l) av[e * 4 + l] = atom_P[e * np + l];
  for (int a = 0; a < h.n_atoms; ++a)
    for (int l = 0; l < np; ++l) ad[a * 4 + l] = atom_D[a * np + l];
  for (int64_t e = 0; e < E; ++e) pr[atom_idx[e] + 1]++;
  for (int64_t i = 0; i < h.N; ++i) pr[i + 1] += pr[i];
  std::vector<int32_t> fill(pr.begin(), pr.end() - 1);
  for (int a = 0; a < h.n_atoms; ++a)
    for (int64_t e = atom_ptr[a]; e < atom_ptr[a + 1]; ++e) {
      const int32_t slot = fill[atom_idx[e]]++;
      for (int l = 0; l < 4; ++l) pv[(int64_t)slot * 4 + l] = av[e * 4 + l];
    }
  upload(h.aval64, av, s);
  upload(h.aD64, ad, s);
  upload(h.pval64, pv, s);
}

// ---------------------------------------------------------------------------------------------
// Persistent autotuning records.  With SCOCG_TUNE_CACHE naming a file, a tuned launch
// shape is appended there as one JSON object per line, keyed by the device
// architecture, precision, grid, nf, atoms, block width, column blocks, energies and
// rows; a later solve of a shape with a record (in any process) takes it instead of
// running the trials.  The library reads only lines in the exact form it writes; the
// last matching record wins; records with values outside the option ranges are
// ignored.  Appends are single write() calls on an O_APPEND descriptor.
struct TuneKey {
  std::string arch;
  int precision, nx, ny, nz, nf, atoms;
  int64_t B, nb, K, nS;
};

std::string tune_key_text(const TuneKey& k) {
  char buf[512];
  snprintf(buf, sizeof buf,
           "{\"arch\": \"%s\", \"precision\": \"%s\", \"grid\": [%d, %d, %d], \"nf\": %d, "
           "\"atoms\": %d, \"block_width\": %lld, \"blocks\": %lld, \"energies\": %lld, "
           "\"rows\": %lld, ",
           k.arch.c_str(), k.precision == SCOCG_FP64 ? "fp64" : "mixed", k.nx, k.ny, k.nz,
           k.nf, k.atoms, (long long)k.B, (long long)k.nb, (long long)k.K, (long long)k.nS);
  return buf;
}

bool tune_record_valid(const std::array<int32_t, 5>& v, int nz) {
  return v[0] >= 1 && v[0] <= 4 && v[1] >= 1 && v[1] <= nz &&
         (v[2] == 1 || v[2] == 4 || v[2] == 16) && v[3] >= 0 && v[3] <= 2 && v[4] >= 0 &&
         v[4] <= nz;
}

bool tune_cache_lookup(const char* path, const TuneKey& k, std::array<int32_t, 5>* out) {
  FILE* f = fopen(path, "r");
  if (!f) return false;
  const std::string key = tune_key_text(k);
  bool found = false;
  char line[1024];
  while (fgets(line, sizeof line, f)) {
    if (strncmp(line, key.c_str(), key.size()) != 0) continue;
    std::array<int32_t, 5> v{};
    char tail = 0;
    if (sscanf(line + key.size(),
               "\"tile\": %d, \"zchunk\": %d, \"shift_chunk\": %d, \"cache_mode\": %d, "
               "\"zchunk_mu\": %d%c",
               &v[0], &v[1], &v[2], &v[3], &v[4], &tail) == 6 &&
        tail == '}' && tune_record_valid(v, k.nz)) {
      *out = v;
      found = true;
    }
  }
  fclose(f);
  return found;
}

void tune_cache_append(const char* path, const TuneKey& k, const std::array<int32_t, 5>& v) {
  char buf[160];
  snprintf(buf, sizeof buf,
           "\"tile\": %d, \"zchunk\": %d, \"shift_chunk\": %d, \"cache_mode\": %d, "
           "\"zchunk_mu\": %d}\n",
           v[0], v[1], v[2], v[3], v[4]);
  const std::string line = tune_key_text(k) + buf;
  const int fd = open(path, O_WRONLY | O_APPEND | O_CREAT, 0644);
  if (fd < 0) {
    if (trace_on()) fprintf(stderr, "[scocg] tune cache %s: cannot open for append\n", path);
    return;
  }
  const ssize_t w = write(fd, line.data(), line.size());
  if (w != (ssize_t)line.size() && trace_on())
    fprintf(stderr, "[scocg] tune cache %s: short write\n", path);
  close(fd);
}

// ---------------------------------------------------------------------------------------------
// complex64 recurrences: a pair is frozen as stalled (and left to refinement) once its
// residual estimate reaches kMixedFloor, near where the FP64 true residual of a
// complex64 solve levels off (measured: 4e-6 median, 4e-5 at the 99th percentile on
// the 16x16x24 grid), or once an estimate below 1e-2 has not halved within
// max(kStallWindow, n/2) iterations
constexpr int kStallWindow = 256;
constexpr double kMixedFloor = 1e-5;

// Solver for one precision: T = vector/stencil arithmetic type, B = columns per block.
template <typename T, int B>
struct Solver {
  using cT = typename cplx_of<T>::type;
  static constexpr int BW = B;
  scocg_ctx& h;
  scocg_ctx::Solve& S;
  explicit Solver(scocg_ctx& hh, scocg_ctx::Solve& ss) : h(hh), S(ss) {}

  // operator arrays in the arithmetic type T: a complex64 handle keeps FP64 copies
  // as well, which an FP64 solver on that handle (refinement escalation) uses
  static constexpr bool DBL = std::is_same<T, double>::value;
  bool use64() const { return DBL && h.precision != SCOCG_FP64; }
  const T* op_vloc() const { return use64() ? h.vloc64.as<T>() : h.vloc.as<T>(); }
  const T* op_aval() const { return use64() ? h.aval64.as<T>() : h.aval.as<T>(); }
  const T* op_aD() const { return use64() ? h.aD64.as<T>() : h.aD.as<T>(); }
  const T* op_pval() const { return use64() ? h.pval64.as<T>() : h.pval.as<T>(); }

  // Krylov vectors: per column block nz + 2*nf planes, nf zero planes on each side
  int64_t pad_points() const { return (int64_t)h.nf * h.nxy; }
  int64_t bstride() const { return ((int64_t)h.nz + 2 * h.nf) * h.nxy * B; }
  // view of a padded vector from its plane 0
  cT* plane0(cT* base) const { return base + pad_points() * B; }

  // stencil workgroup shapes (see scocg_solve_opts::tile)
  struct TileCfg { int tx, ty, nt; };
  static TileCfg tile_cfg(int v) {
    if constexpr (B == 8) {
      switch (v) {
        case 2: return {16, 4, 512};
        case 3: return {8, 8, 512};
        case 4: return {16, 8, 512};
        default: return {16, 8, 1024};
      }
    }
    switch (v) {
      case 2: return {16, 4, 512};
      case 3: return {8, 8, 1024};
      case 4: return {8, 8, 512};
      case 5: return {16, 16, 1024};
      default: return {16, 8, 1024};
    }
  }

  // tiles and z-chunks: as few z-chunks (each re-reads 2*nf planes to fill its
  // queue) as still give `target` workgroups
  StencilGrid plan(int nb, int variant, int zchunk) const {
    // defaults: the spill-free shapes (complex128: 16x8 tile, 1024 threads;
    // complex64: 8x8 tile, 1024 threads)
    if (variant < 1 || variant > 4) variant = B == 8 ? 1 : 3;
    if (h.nf != 4) variant = 1;
    const TileCfg tc = tile_cfg(variant);
    StencilGrid g{};
    g.variant = variant;
    g.ntx = (h.nx + tc.tx - 1) / tc.tx;
    g.nty = (h.ny + tc.ty - 1) / tc.ty;
    const int64_t per_chunk = (int64_t)nb * g.ntx * g.nty;
    // about four groups per CU: shorter z-chunks hide latency better than the
    // re-read of their 2*nf queue planes costs (measured on 48x48x96)
    const int64_t target = (int64_t)256 * 4096 / tc.nt;
    int zc = h.nz;
    if (zchunk > 0) zc = std::min(zchunk, h.nz);
    else
      while (zc > 8 && per_chunk * ((h.nz + zc - 1) / zc) < target) zc = (zc + 1) / 2;
    g.zc = zc;
    g.nzc = (h.nz + zc - 1) / zc;
    g.nwg = g.nzc * g.ntx * g.nty;
    const int64_t total = (int64_t)nb * g.nwg;
    g.nper = (int)((total + 7) / 8);
    g.grid = 8 * g.nper;
    return g;
  }

  // interior-only tiles (the FULL kernels) when the tile divides the plane
  bool full_tiles(int variant) const {
    const TileCfg tc = tile_cfg(h.nf == 4 ? variant : 1);
    return h.nf == 4 && h.nx % tc.tx == 0 && h.ny % tc.ty == 0;
  }

  // x^(k), p^(k) update arguments for workgroups of nth threads, kch energies each
  ShiftArgs<T> shift_args(int nth, int kch) const {
    require(kch >= 1 && kch <= SHIFT_KCH_MAX, "shift chunk outside the staged coefficient range");
    ShiftArgs<T> sa{};
    sa.rnew[0] = to_g(plane0(S.r0.template as<cT>()));
    sa.rnew[1] = to_g(plane0(S.r1.template as<cT>()));
    sa.bstride = bstride();
    sa.srow = S.full ? nullptr : to_g(S.srow.template as<int32_t>());
    sa.nS = S.nS;
    sa.list = to_g(S.list.template as<int32_t>());
    sa.k5cnt = to_g(S.k5cnt.template as<int32_t>());
    sa.K = S.K;
    sa.nb = S.nb;
    sa.coef = to_g(S.coef.template as<ShiftCoef>());
    sa.x = to_g(S.x.template as<double2>());
    sa.p = to_g(S.p.template as<cT>());
    sa.gx = (int)nblocks((int64_t)S.nS * B, nth);
    sa.gy = (int)nblocks(S.K, kch);
    sa.kch = kch;
    sa.sym = S.sym;
    // x (complex128) and p together beyond the 256 MB last-level cache: nontemporal
    const double xp_bytes = (double)S.nb * S.K * S.nS * B * (16.0 + sizeof(cT));
    sa.nt = xp_bytes > 256.0 * (1 << 20);
    return sa;
  }

  // One region's arguments of a stencil pass.  MODE_MU with qa != null also contracts
  // the projectors (into dc and qa) in nproj_wg leading workgroups.  r/io (or the
  // ping-pong pair) are filled by the caller.
  StencilArgs<T> stencil_args(int mode, const StencilGrid& g, int nb, const ColState* cols,
                              const int32_t* blk_active, double2* part0, double* part1, cT* dc,
                              double2* qa) const {
    StencilArgs<T> a{};
    a.bstride = bstride();
    if (mode == MODE_MU && qa && h.n_atoms) {
      a.nproj_wg = (h.n_atoms * nb + 7) / 8 * 8;
      a.proj = proj_args(dc, qa);
    }
    a.vloc = to_g(op_vloc());
    a.co = make_coefs<T>(h);
    a.nx = h.nx; a.ny = h.ny; a.nz = h.nz; a.nxy = h.nxy;
    a.ntx = g.ntx; a.nty = g.nty;
    a.zc = g.zc; a.nzc = g.nzc;
    a.nb = nb;
    a.nper = g.nper;
    a.prow = h.n_atoms ? to_g(h.prow.as<int32_t>()) : nullptr;
    a.patom = to_g(h.patom.as<int32_t>());
    a.pval = to_g(op_pval());
    a.dc = to_g(dc);
    a.n_atoms = h.n_atoms;
    a.cols = to_g(cols);
    a.blk_active = to_g(blk_active);
    a.part0 = to_g(part0);
    a.part1 = to_g(part1);
    return a;
  }

  // workgroups of one region in a stencil launch
  static int stencil_wgs(const StencilArgs<T>& a, const StencilGrid& g) {
    return g.grid + a.nproj_wg + a.nshift_wg;
  }

  // ctl, coff, nctl: control steps run by the first nctl workgroups of a MU launch
  // (none: nctl = 0); n6 = iteration mod 6
  struct CtlIn {
    const ControlArgs* regs = nullptr;
    const int32_t* off = nullptr;
    int n = 0, n6 = 0;
  };

  template <int MODE, int NF, int TX, int TY, int NT>
  static void launch_v(hipStream_t st, bool full, const StencilArgs<T>* regs, const int32_t* off,
                       int nreg, int grid, int cur, CtlIn ci) {
    if (full && NF == 4)
      hipLaunchKernelGGL((k_stencil<T, NF, B, MODE, TX, TY, NT, true>), dim3(grid + ci.n),
                         dim3(NT), 0, st, regs, off, nreg, cur, ci.regs, ci.off, ci.n, ci.n6);
    else
      hipLaunchKernelGGL((k_stencil<T, NF, B, MODE, TX, TY, NT, false>), dim3(grid + ci.n),
                         dim3(NT), 0, st, regs, off, nreg, cur, ci.regs, ci.off, ci.n, ci.n6);
  }

  // one stencil launch over a device table of nreg regions (common nf, tile variant)
  template <int MODE>
  static void launch_table(hipStream_t st, int nf, int variant, bool full,
                           const StencilArgs<T>* regs, const int32_t* off, int nreg, int grid,
                           int cur, CtlIn ci = CtlIn()) {
    switch (nf) {
      case 1: launch_v<MODE, 1, 16, 8, 1024>(st, full, regs, off, nreg, grid, cur, ci); break;
      case 2: launch_v<MODE, 2, 16, 8, 1024>(st, full, regs, off, nreg, grid, cur, ci); break;
      case 3: launch_v<MODE, 3, 16, 8, 1024>(st, full, regs, off, nreg, grid, cur, ci); break;
      default:
        if constexpr (B == 8) {
          switch (variant) {
            case 2: launch_v<MODE, 4, 16, 4, 512>(st, full, regs, off, nreg, grid, cur, ci); break;
            case 3: launch_v<MODE, 4, 8, 8, 512>(st, full, regs, off, nreg, grid, cur, ci); break;
            case 4: launch_v<MODE, 4, 16, 8, 512>(st, full, regs, off, nreg, grid, cur, ci); break;
            default: launch_v<MODE, 4, 16, 8, 1024>(st, full, regs, off, nreg, grid, cur, ci); break;
          }
        } else {
          switch (variant) {
            case 2: launch_v<MODE, 4, 16, 4, 512>(st, full, regs, off, nreg, grid, cur, ci); break;
            case 3: launch_v<MODE, 4, 8, 8, 1024>(st, full, regs, off, nreg, grid, cur, ci); break;
            case 4: launch_v<MODE, 4, 8, 8, 512>(st, full, regs, off, nreg, grid, cur, ci); break;
            default: launch_v<MODE, 4, 16, 8, 1024>(st, full, regs, off, nreg, grid, cur, ci); break;
          }
        }
    }
    KCHK();
  }

  ProjArgs<T> proj_args(cT* dc, double2* qa) const {
    ProjArgs<T> pa{};
    pa.aptr = to_g(h.aptr.as<int32_t>());
    pa.aidx = to_g(h.aidx.as<int32_t>());
    pa.aval = to_g(op_aval());
    pa.aD = to_g(op_aD());
    pa.n_proj = h.n_proj;
    pa.n_atoms = h.n_atoms;
    pa.dc = to_g(dc);
    pa.qa = to_g(qa);
    pa.mfma = h.proj_mfma;
    return pa;
  }

  // r: padded vector base
  void launch_proj(cT* r, int nb, cT* dc, const int32_t* blk_active) {
    if (!h.n_atoms) return;
    hipLaunchKernelGGL((k_proj<T, B>), dim3(h.n_atoms, nb), dim3(WG), 0, h.stream, plane0(r),
                       bstride(), proj_args(dc, nullptr), blk_active);
    KCHK();
  }

  // dynamic LDS of k_control: |pi| (double) and an activity byte per (shift, column)
  static size_t control_lds(int K) { return (size_t)K * B * (sizeof(double) + 1); }

  // FP64 operator data (the handle's own arrays for SCOCG_FP64, the FP64 copies otherwise)
  const double* vloc64() const {
    return h.precision == SCOCG_FP64 ? h.vloc.as<double>() : h.vloc64.as<double>();
  }
  ProjArgs<double> proj64(double2* dc) const {
    const bool f = h.precision == SCOCG_FP64;
    ProjArgs<double> pa{};
    pa.aptr = to_g(h.aptr.as<int32_t>());
    pa.aidx = to_g(h.aidx.as<int32_t>());
    pa.aval = to_g(f ? h.aval.as<double>() : h.aval64.as<double>());
    pa.aD = to_g(f ? h.aD.as<double>() : h.aD64.as<double>());
    pa.n_proj = h.n_proj;
    pa.n_atoms = h.n_atoms;
    pa.dc = to_g(dc);
    pa.qa = nullptr;
    return pa;
  }

  // FP64 ||e_j - (z_k - H) x^(k)_j|| for every pair of a full-storage solve
  // (x in [nb*K][N][B]); t is kept in `tbuf` when it is non-null.  Returns the
  // norms as [nb*K*B] (block kb = cb*K + k, column c).
  std::vector<double> true_residuals(DevBuf* tbuf) {
    const int nblk = S.nb * S.K;
    const int64_t N = h.N;
    constexpr int PTS = WG / B;
    const int gx = (int)nblocks(N, PTS);
    DevBuf part, norms, dc64;
    part.alloc((size_t)nblk * gx * B * sizeof(double));
    norms.alloc((size_t)nblk * B * sizeof(double));
    if (h.n_atoms) {
      dc64.alloc((size_t)nblk * h.n_atoms * 4 * B * sizeof(double2));
      hipLaunchKernelGGL((k_proj<double, B>), dim3(h.n_atoms, nblk), dim3(WG), 0, h.stream,
                         S.x.as<double2>(), N * B, proj64(dc64.as<double2>()), nullptr);
      KCHK();
    }
    if (tbuf) tbuf->alloc((size_t)nblk * N * B * sizeof(double2));
    const Coefs<double> co = make_coefs<double>(h);
    const dim3 g(gx, nblk);
    const double2* x = S.x.as<double2>();
    double2* t = tbuf ? tbuf->as<double2>() : nullptr;
    const int32_t* prow = h.n_atoms ? h.prow.as<int32_t>() : nullptr;
    const double* pv = h.n_atoms ? (h.precision == SCOCG_FP64 ? h.pval.as<double>()
                                                               : h.pval64.as<double>())
                                 : nullptr;
#define SCOCG_TR(NFV)                                                                         \
  hipLaunchKernelGGL((k_true_resid<NFV, B>), g, dim3(WG), 0, h.stream, x, t, vloc64(), co, h.nx, \
                     h.ny, h.nz, prow, h.patom.as<int32_t>(), pv, dc64.as<double2>(),          \
                     h.n_atoms, S.z.as<double2>(), S.rhs.as<int32_t>(), S.R, S.K,              \
                     part.as<double>())
    switch (h.nf) {
      case 1: SCOCG_TR(1); break;
      case 2: SCOCG_TR(2); break;
      case 3: SCOCG_TR(3); break;
      default: SCOCG_TR(4); break;
    }
#undef SCOCG_TR
    KCHK();
    hipLaunchKernelGGL((k_norms<B>), dim3(nblk), dim3(WG), 0, h.stream, part.as<double>(), gx,
                       norms.as<double>());
    KCHK();
    std::vector<double> out((size_t)nblk * B);
    HIPCHK(hipMemcpyAsync(out.data(), norms.p, out.size() * sizeof(double), hipMemcpyDeviceToHost,
                          h.stream));
    HIPCHK(hipStreamSynchronize(h.stream));
    return out;
  }

  // ---- solve state
  void alloc_state(int K, int R, bool full, int nS, const scocg_solve_opts& o) {
    require((R + B - 1) / B <= 65536, "too many column blocks");
    require(control_lds(K) <= 128 * 1024, "too many energies for one column block (K*B)");
    HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_control<B>),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)control_lds(K)));
    S.B = B;
    S.K = K;
    S.R = R;
    S.nb = (R + B - 1) / B;
    S.full = full;
    S.nS = nS;
    const int nb = S.nb;
    S.g = plan(nb, o.tile, o.zchunk);
    S.nwg = S.g.nwg;
    S.kch = o.shift_chunk > 0 ? o.shift_chunk : 4;
    S.cache_mode = o.cache_mode > 0 ? o.cache_mode : 0;
    S.zc_mu = o.zchunk_mu > 0 ? o.zchunk_mu : 0;
    const size_t vec = (size_t)nb * bstride() * sizeof(cT);
    S.r0.alloc(vec);
    S.r1.alloc(vec);
    const size_t nkb = (size_t)nb * K * B;
    S.z.alloc(nkb * sizeof(double2));
    S.sh.alloc(nkb * sizeof(ShiftState));
    S.coef.alloc(2 * nkb * sizeof(ShiftCoef));  // by iteration parity
    S.cols.alloc((size_t)nb * B * sizeof(ColState));
    S.list.alloc((size_t)3 * nb * K * sizeof(int32_t));  // iteration n: n mod 3
    S.cnt.alloc((size_t)3 * nb * sizeof(int32_t));
    S.k5cnt.alloc((size_t)2 * nb * sizeof(int32_t));
    S.pim.alloc(nkb * sizeof(double));  // control scratch inside the mu launch
    S.act.alloc(nkb);
    S.blk_active.alloc((size_t)nb * sizeof(int32_t));
    S.blk_iter.alloc((size_t)nb * sizeof(int32_t));
    const size_t xp = nkb * (size_t)S.nS;
    S.x.alloc(xp * sizeof(double2));
    S.p.alloc(xp * sizeof(cT));
    S.dc.alloc((size_t)std::max(h.n_atoms, 1) * nb * 4 * B * sizeof(cT));
    S.qa.alloc((size_t)std::max(h.n_atoms, 1) * nb * B * sizeof(double2));
    // rho / ||r||^2 partials of the r_{n+1} pass, and the mu pass's own (the control
    // step of n - 1 reads the former while the mu pass of n writes the latter)
    S.part0.alloc((size_t)nb * S.nwg * B * sizeof(double2));
    S.part1.alloc((size_t)nb * S.nwg * B * sizeof(double));
    S.partm.alloc((size_t)nb * mu_grid().nwg * B * sizeof(double2));
    if (!S.h_flags) HIPCHK(hipHostMalloc((void**)&S.h_flags, sizeof(int32_t) * 65536));
  }

  // unit right-hand sides e_{rhs[j]}, energies zk[K] shared by every column
  // zpc (K == 1 only): one energy per column instead of zk[K] shared by all columns
  void init_unit(const double2* zk, int seed0, const double2* zpc = nullptr) {
    hipStream_t st = h.stream;
    const int nb = S.nb, K = S.K, R = S.R;
    const size_t nkb = (size_t)nb * K * B;
    hipLaunchKernelGGL((k_init_r<T, B>), dim3(nblocks((int64_t)nb * bstride(), WG)), dim3(WG), 0,
                       st, S.r0.as<cT>(), S.r1.as<cT>(), bstride(), h.N, pad_points(),
                       S.rhs.as<int32_t>(), R, nb);
    KCHK();
    hipLaunchKernelGGL((k_init_xp<T, B>), dim3(nblocks((int64_t)nkb * S.nS, WG)), dim3(WG), 0, st,
                       S.x.as<double2>(), S.p.as<cT>(), S.full ? nullptr : S.srow.as<int32_t>(),
                       S.nS, K, nb, S.rhs.as<int32_t>(), R);
    KCHK();
    hipLaunchKernelGGL((k_init_state<B>), dim3(nblocks((int64_t)nkb, WG)), dim3(WG), 0, st,
                       S.cols.as<ColState>(), S.sh.as<ShiftState>(), S.coef.as<ShiftCoef>(),
                       S.z.as<double2>(), zk, zpc, nullptr, K, nb, R, seed0, S.list.as<int32_t>(),
                       S.cnt.as<int32_t>(), S.k5cnt.as<int32_t>(), S.blk_active.as<int32_t>(),
                       S.blk_iter.as<int32_t>());
    KCHK();
  }

  // dense right-hand sides (K = 1, full storage): column j solves
  // (zpc[j] - H) d = scale[j] * src[src_kb[j]][:][src_c[j]]
  template <int BS>
  void init_dense(const double2* zpc, const double2* src, const int32_t* src_kb,
                  const int32_t* src_c, const double* scale, const double* tolc) {
    hipStream_t st = h.stream;
    const int nb = S.nb, R = S.R;
    const int gx = (int)nblocks(bstride(), WG);
    DevBuf prho, pnu;
    prho.alloc((size_t)nb * gx * B * sizeof(double2));
    pnu.alloc((size_t)nb * gx * B * sizeof(double));
    hipLaunchKernelGGL((k_init_r_dense<T, B, BS>), dim3(gx, nb), dim3(WG), 0, st, S.r0.as<cT>(),
                       S.r1.as<cT>(), bstride(), h.N, pad_points(), src, src_kb, src_c, scale, R,
                       prho.as<double2>(), pnu.as<double>());
    KCHK();
    hipLaunchKernelGGL((k_init_xp_dense<T, B>), dim3(nblocks((int64_t)nb * h.N * B, WG)), dim3(WG),
                       0, st, S.x.as<double2>(), S.p.as<cT>(), plane0(S.r0.as<cT>()), bstride(),
                       h.N, nb);
    KCHK();
    hipLaunchKernelGGL((k_init_state<B>), dim3(nblocks((int64_t)nb * B, WG)), dim3(WG), 0, st,
                       S.cols.as<ColState>(), S.sh.as<ShiftState>(), S.coef.as<ShiftCoef>(),
                       S.z.as<double2>(), zpc, zpc, tolc, 1, nb, R, 0, S.list.as<int32_t>(),
                       S.cnt.as<int32_t>(), S.k5cnt.as<int32_t>(), S.blk_active.as<int32_t>(),
                       S.blk_iter.as<int32_t>());
    KCHK();
    hipLaunchKernelGGL((k_dense_cols<B>), dim3(nb), dim3(WG), 0, st, prho.as<double2>(),
                       pnu.as<double>(), gx, S.cols.as<ColState>(), R);
    KCHK();
    HIPCHK(hipStreamSynchronize(st));  // prho, pnu are freed on return
  }

  // the seed iterations of this solve alone (a batch of one region)
  int64_t iterate(const scocg_solve_opts& o, double* kms, int64_t* kcount);

  // switch the stencil launch shape, growing the partial-sum buffers if needed
  void set_grid(const StencilGrid& g) {
    S.g = g;
    S.nwg = g.nwg;
    fit_partials();
  }

  // launch shape of the mu pass: the r_{n+1} pass's tile with its own z-chunk
  StencilGrid mu_grid() const {
    return S.zc_mu > 0 && S.zc_mu != S.g.zc ? plan(S.nb, S.g.variant, S.zc_mu) : S.g;
  }

  void set_mu_zchunk(int zc) {
    S.zc_mu = zc;
    fit_partials();
  }

  // partial-sum buffers for both passes' workgroup counts
  void fit_partials() {
    const size_t need = (size_t)S.nb * S.g.nwg * B;
    const size_t need_mu = (size_t)S.nb * mu_grid().nwg * B;
    if (S.part0.bytes < need * sizeof(double2)) S.part0.alloc(need * sizeof(double2));
    if (S.part1.bytes < need * sizeof(double)) S.part1.alloc(need * sizeof(double));
    if (S.partm.bytes < need_mu * sizeof(double2)) S.partm.alloc(need_mu * sizeof(double2));
  }

  // Device time per seed iteration of `iters` iterations from the initial state
  double trial(const double2* zk, int seed0, const scocg_solve_opts& o, int iters) {
    scocg_solve_opts ot = o;
    ot.max_iter = iters;
    ot.timing = 0;
    ot.use_graph = 0;
    ot.poll_every = iters;
    init_unit(zk, seed0, conv ? zk : nullptr);
    Event a, b;
    HIPCHK(hipEventRecord(a, h.stream));
    double km[SCOCG_K_FAMILIES] = {0};
    int64_t kc[SCOCG_K_FAMILIES] = {0};
    const int64_t n = iterate(ot, km, kc);
    HIPCHK(hipEventRecord(b, h.stream));
    return 1e3 * elapsed_ms(a, b) / (double)std::max<int64_t>(n, 1);
  }

  // Autotuning: time each candidate stencil shape (tile x z-chunk), then each shift
  // chunk, on this problem; keep the fastest.  Returns the device time spent.
  double tune(const double2* zk, int seed0, const scocg_solve_opts& o, bool want_tile,
              bool want_zc, bool want_kch, bool want_cache, bool want_zc_mu) {
    constexpr int kIters = 16;
    Event a, b;
    HIPCHK(hipEventRecord(a, h.stream));
    if (want_tile || want_zc) {
      std::vector<int> vs;
      if (want_tile && h.nf == 4) vs = {1, 2, 3, 4};
      else vs = {want_tile ? 1 : std::max(o.tile, 0)};
      double best = INFINITY;
      StencilGrid bg = S.g;
      for (int v : vs) {
        const StencilGrid g0 = plan(S.nb, v, want_zc ? 0 : o.zchunk);
        std::vector<int> zcs = {g0.zc};
        // shorter chunks re-read more queue planes but keep the tiles of a chunk
        // marching closer together (halo reads that hit L2); longer ones the reverse
        if (want_zc)
          for (int zc : {g0.zc / 8, g0.zc / 4, g0.zc / 2, g0.zc * 4 / 3, g0.zc * 3 / 2,
                         g0.zc * 2, g0.zc * 4})
            if (zc >= 6 && zc <= h.nz) zcs.push_back(zc);
        std::sort(zcs.begin(), zcs.end());
        zcs.erase(std::unique(zcs.begin(), zcs.end()), zcs.end());
        for (int zc : zcs) {
          const StencilGrid g = plan(S.nb, v, zc);
          set_grid(g);
          const double us = trial(zk, seed0, o, kIters);
          if (trace_on())
            fprintf(stderr, "[scocg] tune tile %d zchunk %d: %.1f us/iteration\n", g.variant,
                    g.zc, us);
          if (us < best) {
            best = us;
            bg = g;
          }
        }
      }
      set_grid(bg);
    }
    if (want_zc_mu) {
      // the mu pass runs two workgroups per CU and reads only a one-sided halo: longer
      // chunks (fewer queue refills) may pay there while the r_{n+1} pass keeps its own
      const int zc = S.g.zc;
      std::vector<int> zcs = {0};
      for (int c : {zc * 4 / 3, zc * 3 / 2, zc * 2, zc * 3, h.nz})
        if (c > zc && c <= h.nz) zcs.push_back(c);
      std::sort(zcs.begin() + 1, zcs.end());
      zcs.erase(std::unique(zcs.begin() + 1, zcs.end()), zcs.end());
      double best = INFINITY;
      int bz = 0;
      for (int c : zcs) {
        set_mu_zchunk(c);
        const double us = trial(zk, seed0, o, kIters);
        if (trace_on())
          fprintf(stderr, "[scocg] tune mu zchunk %d: %.1f us/iteration\n", mu_grid().zc, us);
        if (us < best) {
          best = us;
          bz = c;
        }
      }
      set_mu_zchunk(bz);
    }
    if (want_kch) {
      double best = INFINITY;
      int bk = 4;
      for (int kch : {1, 4, 16}) {
        S.kch = kch;
        const double us = trial(zk, seed0, o, kIters);
        if (trace_on()) fprintf(stderr, "[scocg] tune shift chunk %d: %.1f us/iteration\n", kch, us);
        if (us < best) {
          best = us;
          bk = kch;
        }
      }
      S.kch = bk;
    }
    if (want_cache) {
      // whole-iteration effect of the r_{n+1} pass's cache policy: nontemporal streams
      // keep r_n's halo planes in cache within the pass; ordinary stores leave r_{n+1}
      // in the last-level cache for the mu pass that reads it next
      double best = INFINITY;
      int bm = 0;
      for (int m : {0, 1, 2}) {
        S.cache_mode = m;
        const double us = trial(zk, seed0, o, kIters);
        if (trace_on()) fprintf(stderr, "[scocg] tune cache mode %d: %.1f us/iteration\n", m, us);
        if (us < best) {
          best = us;
          bm = m;
        }
      }
      S.cache_mode = bm;
    }
    HIPCHK(hipEventRecord(b, h.stream));
    return elapsed_ms(a, b);
  }

  void release_workspace() {
    S.r0.release();
    S.r1.release();
    S.part0.release();
    S.part1.release();
    S.partm.release();
    S.pim.release();
    S.act.release();
    S.dc.release();
    S.qa.release();
  }

  // One correction pass with an inner solver of type SolverIn: every pair whose
  // FP64 true residual misses tol gets a single-energy COCG solve of
  // (z_k - H) d = t / ||t|| (at most `cap` iterations) and x += ||t|| d in FP64.
  // Returns the number of pairs corrected; tres (in/out) holds the true
  // residuals ([nb*K*B] layout).
  template <typename SolverIn>
  int64_t correction_pass(const scocg_solve_opts& o, int pass, int64_t cap, const double2* zk_host,
                          std::vector<double>& tres) {
    constexpr int BI = SolverIn::BW;
    std::vector<int32_t> kb, cc;
    std::vector<double> sc, back, tolc;
    std::vector<double2> zp;
    double tmax = 0.0;
    for (int cb = 0; cb < S.nb; ++cb)
      for (int k = 0; k < S.K; ++k)
        for (int c = 0; c < B; ++c) {
          const double t = tres[((size_t)cb * S.K + k) * B + c];
          if (cb * B + c >= S.R || !(t > o.tol)) continue;
          kb.push_back(cb * S.K + k);
          cc.push_back(c);
          sc.push_back(1.0 / t);
          back.push_back(t);
          // the corrected residual is ||t|| times the inner relative residual
          tolc.push_back(std::min(0.5, std::max(1e-12, 0.25 * o.tol / t)));
          zp.push_back(conv ? zcol[(size_t)cb * B + c] : zk_host[k]);
          tmax = std::max(tmax, t);
        }
    if (kb.empty()) return 0;
    const int Rin = (int)kb.size();
    DevBuf d_kb, d_c, d_sc, d_back, d_z, d_tol, tbuf;
    tres = true_residuals(&tbuf);  // the residual vectors themselves
    upload(d_kb, kb, h.stream);
    upload(d_c, cc, h.stream);
    upload(d_sc, sc, h.stream);
    upload(d_back, back, h.stream);
    upload(d_tol, tolc, h.stream);
    // per-column energies of the inner solve, padded to whole blocks
    zp.resize((size_t)((Rin + BI - 1) / BI) * BI, zp.back());
    upload(d_z, zp, h.stream);
    scocg_ctx::Solve Sin;
    SolverIn in(h, Sin);
    scocg_solve_opts oi = o;
    oi.full = 1;
    oi.init_seed = 0;
    oi.tile = 0;
    oi.zchunk = 0;
    oi.shift_chunk = 0;
    oi.max_iter = cap;
    oi.tol = std::min(0.5, std::max(1e-12, 0.25 * o.tol / tmax));  // per-column tolc rules
    oi.timing = 0;
    in.alloc_state(1, Rin, true, (int)h.N, oi);
    in.template init_dense<B>(d_z.as<double2>(), tbuf.as<double2>(), d_kb.as<int32_t>(),
                              d_c.as<int32_t>(), d_sc.as<double>(), d_tol.as<double>());
    double km[SCOCG_K_FAMILIES] = {0};
    int64_t kc[SCOCG_K_FAMILIES] = {0};
    const int64_t it_in = in.iterate(oi, km, kc);
    if (trace_on()) {
      std::vector<ShiftState> si((size_t)Sin.nb * BI);
      HIPCHK(hipMemcpy(si.data(), Sin.sh.p, si.size() * sizeof(ShiftState), hipMemcpyDeviceToHost));
      int conv = 0, brk = 0;
      double emax = 0;
      for (int j = 0; j < Rin; ++j) {
        conv += si[j].status == ST_CONVERGED && !si[j].active;
        brk += si[j].status == ST_BREAKDOWN;
        emax = std::max(emax, si[j].est);
      }
      fprintf(stderr,
              "[scocg] correction pass %d (%s inner): %d pairs, max true residual %.3e, inner "
              "tol %.3e, %lld inner iterations, %d converged, %d breakdown, max est %.3e\n",
              pass, BI == 8 ? "complex128" : "complex64", Rin, tmax, oi.tol, (long long)it_in,
              conv, brk, emax);
    }
    hipLaunchKernelGGL((k_add_correction<BI, B>), dim3(nblocks((int64_t)Rin * h.N, WG)), dim3(WG),
                       0, h.stream, S.x.as<double2>(), Sin.x.as<double2>(), d_kb.as<int32_t>(),
                       d_c.as<int32_t>(), d_back.as<double>(), Sin.sh.as<ShiftState>(), Rin,
                       h.N);
    KCHK();
    tbuf.release();
    tres = true_residuals(nullptr);
    return Rin;
  }

  // Refinement of a full-storage complex64 solve: up to `passes` correction
  // passes with complex64 inner solves (each capped at twice the outer seed
  // iterations, since plain FP32 COCG can stall on the hardest energies), then
  // one pass with complex128 inner solves for the pairs still above tol.
  int64_t refine(const scocg_solve_opts& o, int passes, int64_t outer_iters,
                 const double2* zk_host, std::vector<double>& tres) {
    int64_t refined = 0;
    const int64_t cap = std::max<int64_t>(outer_iters, 200);
    auto worst = [&]() {
      double m = 0.0;
      for (int cb = 0; cb < S.nb; ++cb)
        for (int k = 0; k < S.K; ++k)
          for (int c = 0; c < B && cb * B + c < S.R; ++c)
            m = std::max(m, tres[((size_t)cb * S.K + k) * B + c]);
      return m;
    };
    for (int pass = 0; pass < passes; ++pass) {
      const double before = worst();
      const int64_t n = correction_pass<Solver<T, B>>(o, pass, cap, zk_host, tres);
      refined += n;
      // stop the complex64 passes once they stall (worst residual not cut 10x)
      if (!n || worst() > 0.1 * before) break;
    }
    if constexpr (!DBL) refined += correction_pass<Solver<double, 8>>(o, passes, 4 * cap, zk_host, tres);
    return refined;
  }

  // ---- phases of a solve (a batch runs the same phases around one shared iteration loop)
  std::vector<double2> zh;  // energies (host copy)
  DevBuf zk;                // energies on the device (conventional: one per column)
  int seed0 = 0;
  bool conv = false;              // conventional sweep: column k*R + j solves (z_k - H) x = e_j
  std::vector<double2> zcol;      // conventional: energy of every column (padded to whole blocks)

  // inputs and state; no kernel of the solve proper yet
  void prepare(int K, const double* z, int R, const int64_t* rhs_idx, int nS_in,
               const int64_t* s_idx, const scocg_solve_opts& o) {
    const bool full = o.full != 0;
    const int nS = full ? (int)h.N : (s_idx ? nS_in : R);
    hipStream_t st = h.stream;
    zh.resize(K);
    for (int k = 0; k < K; ++k) zh[k] = mk(z[2 * k], z[2 * k + 1]);
    std::vector<int32_t> rh(R);
    for (int j = 0; j < R; ++j) rh[j] = (int32_t)rhs_idx[j];
    upload(S.rhs, rh, st);
    if (!full) {
      std::vector<int32_t> sr(nS);
      for (int i = 0; i < nS; ++i) sr[i] = (int32_t)(s_idx ? s_idx[i] : rhs_idx[i]);
      upload(S.srow, sr, st);
    }
    conv = o.conventional != 0;
    S.sym = o.symmetric;
    if (!conv) {
      // an auxiliary seed energy is one more shift after the K returned ones
      const int Kt = o.aux_seed ? K + 1 : K;
      if (o.aux_seed) zh.push_back(mk(o.seed_z[0], o.seed_z[1]));
      upload(zk, zh, st);
      alloc_state(Kt, R, full, nS, o);
      S.Kout = K;
      seed0 = o.aux_seed ? K : (o.init_seed < 0 ? K / 2 : o.init_seed);
      return;
    }
    // conventional sweep: K*R single-energy systems, column k*R + j = (z_k, e_{rhs_j}); the
    // report and output layouts [1][K*R] and [1][K*R][nS] are those of [K][R] and [K][R][nS]
    const int64_t RC = (int64_t)K * R;
    require(RC <= INT32_MAX / B, "too many (energy, column) pairs for the conventional sweep");
    std::vector<int32_t> rc((size_t)RC);
    zcol.assign((size_t)((RC + B - 1) / B) * B, zh[K - 1]);
    for (int k = 0; k < K; ++k)
      for (int j = 0; j < R; ++j) {
        rc[(size_t)k * R + j] = rh[j];
        zcol[(size_t)k * R + j] = zh[k];
      }
    upload(S.rhs, rc, st);
    upload(zk, zcol, st);
    alloc_state(1, (int)RC, full, nS, o);
    S.Kout = 1;
    seed0 = 0;
  }

  // autotuning (outside the timed region; cached per shape in the handle)
  double autotune(const scocg_solve_opts& o, int* tuned_now) {
    *tuned_now = 0;
    const bool auto_tile = o.tile == SCOCG_AUTO, auto_zc = o.zchunk == SCOCG_AUTO,
               auto_kch = o.shift_chunk == SCOCG_AUTO, auto_cache = o.cache_mode == SCOCG_AUTO,
               auto_zc_mu = o.zchunk_mu == SCOCG_AUTO;
    if (!(auto_tile || auto_zc || auto_kch || auto_cache || auto_zc_mu)) return 0.0;
    const std::array<int64_t, 4> key{B, S.nb, S.K, S.nS};
    auto it = h.tuned.find(key);
    const char* file = getenv("SCOCG_TUNE_CACHE");
    const bool use_file = file && *file;
    const TuneKey tk{h.arch, h.precision, h.nx, h.ny, h.nz, h.nf, h.n_atoms, B, S.nb, S.K, S.nS};
    if (it == h.tuned.end() && use_file) {
      std::array<int32_t, 5> rec{};
      if (tune_cache_lookup(file, tk, &rec)) it = h.tuned.emplace(key, rec).first;
    }
    if (it != h.tuned.end()) {
      set_grid(plan(S.nb, auto_tile ? it->second[0] : o.tile, auto_zc ? it->second[1] : o.zchunk));
      if (auto_kch) S.kch = it->second[2];
      if (auto_cache) S.cache_mode = it->second[3];
      if (auto_zc_mu) set_mu_zchunk(it->second[4]);
      return 0.0;
    }
    const double ms = tune(zk.as<double2>(), seed0, o, auto_tile, auto_zc, auto_kch,
                           auto_cache, auto_zc_mu);
    *tuned_now = 1;
    h.tuned[key] = {S.g.variant, S.g.zc, S.kch, S.cache_mode, S.zc_mu};
    if (use_file) tune_cache_append(file, tk, h.tuned[key]);
    return ms;
  }

  // after the iterations: trace, FP64 true residuals (full storage) and, for complex64,
  // refinement; all inside the timed region
  int64_t post(const scocg_solve_opts& o, int64_t it_main, std::vector<double>& tres) {
    const size_t nkb = (size_t)S.nb * S.K * B;
    release_workspace();
    if (trace_on()) {
      std::vector<ShiftState> s0(nkb);
      HIPCHK(hipMemcpy(s0.data(), S.sh.p, nkb * sizeof(ShiftState), hipMemcpyDeviceToHost));
      int64_t n_st[5] = {0, 0, 0, 0, 0};
      for (const auto& x : s0) n_st[x.active ? ST_MAXITER : std::min(std::max(x.status, 0), 4)]++;
      fprintf(stderr,
              "[scocg] main solve: %lld iterations; pairs converged %lld, max-iter %lld, "
              "breakdown %lld, stalled %lld\n",
              (long long)it_main, (long long)n_st[0], (long long)n_st[1], (long long)n_st[2],
              (long long)n_st[4]);
    }
    int64_t refined = 0;
    if (S.full && o.refine >= 0) {
      tres = true_residuals(nullptr);
      if (h.precision == SCOCG_MIXED && o.refine > 0) {
        int32_t mx = 0;
        std::vector<ColState> c0((size_t)S.nb * B);
        HIPCHK(hipMemcpy(c0.data(), S.cols.p, c0.size() * sizeof(ColState), hipMemcpyDeviceToHost));
        for (int j = 0; j < S.R; ++j) mx = std::max(mx, c0[j].iters);
        refined = refine(o, o.refine, mx, zh.data(), tres);
      }
    }
    return refined;
  }

  // fills the report; returns the solve's return code
  int report(const scocg_solve_opts& o, const std::vector<double>& tres, int64_t refined, float ms,
             const double* kms, const int64_t* kcount, double tune_ms, int tuned_now,
             scocg_report* rep) {
    const int nb = S.nb, K = S.K, R = S.R;
    const size_t nkb = (size_t)nb * K * B;
    std::vector<ShiftState> shh(nkb);
    std::vector<ColState> ch((size_t)nb * B);
    std::vector<int32_t> bit(nb);
    HIPCHK(hipMemcpy(bit.data(), S.blk_iter.p, nb * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(shh.data(), S.sh.p, nkb * sizeof(ShiftState), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(ch.data(), S.cols.p, ch.size() * sizeof(ColState), hipMemcpyDeviceToHost));
    int rc = SCOCG_OK;
    int64_t seed_iters = 0, nsw = 0;
    for (int j = 0; j < R; ++j) {
      seed_iters = std::max<int64_t>(seed_iters, ch[j].iters);
      nsw += ch[j].nswitch;
    }
    for (int k = 0; k < S.Kout; ++k)
      for (int j = 0; j < R; ++j) {
        const size_t so = ((size_t)(j / B) * K + k) * B + (j % B);
        const ShiftState& ss = shh[so];
        int stt = ss.status;
        if (ss.active) stt = ST_MAXITER;
        // complex64 vectors: the FP64 true residual, where computed, decides
        if (!DBL && !tres.empty() && stt != ST_BREAKDOWN)
          stt = tres[so] <= o.tol ? ST_CONVERGED : (stt == ST_MAXITER ? ST_MAXITER : ST_STALLED);
        if (stt != ST_CONVERGED && stt != ST_BREAKDOWN && rc == SCOCG_OK)
          rc = SCOCG_NOT_ALL_CONVERGED;
        if (stt == ST_BREAKDOWN) rc = SCOCG_BREAKDOWN;
        const size_t o2 = (size_t)k * R + j;
        if (rep) {
          if (rep->iters) rep->iters[o2] = ss.iters;
          if (rep->est_resid) rep->est_resid[o2] = ss.est;
          if (rep->true_resid) rep->true_resid[o2] = tres.empty() ? NAN : tres[so];
          if (rep->status) rep->status[o2] = stt;
        }
      }
    if (rep) {
      rep->seed_iters = seed_iters;
      rep->n_switches = nsw;
      rep->refined = refined;
      rep->solve_ms = ms;
      rep->block_iters = 0;
      for (int b = 0; b < nb; ++b) rep->block_iters += bit[b];
      rep->block_width = B;
      rep->n_blocks = nb;
      for (int f = 0; f < SCOCG_K_FAMILIES; ++f) {
        rep->kernel_ms[f] = kms[f];
        rep->kernel_launches[f] = kcount[f];
      }
      rep->tile_used = S.g.variant;
      rep->zchunk_used = S.g.zc;
      rep->shift_chunk_used = S.kch;
      rep->cache_mode_used = S.cache_mode;
      rep->zchunk_mu_used = mu_grid().zc;
      rep->tuned = tuned_now;
      rep->tune_ms = tune_ms;
    }
    S.ok = true;
    return rc;
  }

  int run(int K, const double* z, int R, const int64_t* rhs_idx, int nS_in, const int64_t* s_idx,
          const scocg_solve_opts& o, scocg_report* rep) {
    hipStream_t st = h.stream;
    prepare(K, z, R, rhs_idx, nS_in, s_idx, o);
    int tuned_now = 0;
    const double tune_ms = autotune(o, &tuned_now);
    Event e0, e1;
    HIPCHK(hipEventRecord(e0, st));
    init_unit(zk.as<double2>(), seed0, conv ? zk.as<double2>() : nullptr);
    double kms[SCOCG_K_FAMILIES] = {0};
    int64_t kcount[SCOCG_K_FAMILIES] = {0};
    const int64_t it_main = iterate(o, kms, kcount);
    std::vector<double> tres;
    const int64_t refined = post(o, it_main, tres);
    HIPCHK(hipEventRecord(e1, st));
    const float ms = elapsed_ms(e0, e1);
    return report(o, tres, refined, ms, kms, kcount, tune_ms, tuned_now, rep);
  }
};

// Seed iterations of one or more regions (solvers of one precision on one stream,
// same nf, tile variant and shift chunk): every kernel family is ONE launch per
// iteration over a device table of per-region arguments; the host polls every
// region's block flags every `poll` iterations, and the polled iterations can be
// replayed as one captured hipGraph.
template <typename T, int B>
struct Batch {
  using SV = Solver<T, B>;
  using cT = typename cplx_of<T>::type;
  std::vector<SV*> sv;
  hipStream_t st = nullptr;
  int nf = 4, variant = 1, kch = 4;
  bool full = true;
  DevBuf t_mu, t_upd, t_alpha, t_ctl, t_shift, o_mu, o_upd, o_blk, o_shift;
  int g_mu = 0, g_upd = 0, g_blk = 0, g_shift = 0;
  size_t ctl_lds = 0;
  int timing_mode = 0;

  Batch(std::vector<SV*> v, const scocg_solve_opts& o) : sv(std::move(v)) {
    require(!sv.empty(), "empty batch");
    const SV& s0 = *sv[0];
    st = s0.h.stream;
    nf = s0.h.nf;
    variant = s0.S.g.variant;
    kch = s0.S.kch;
    std::vector<StencilArgs<T>> mu, up;
    std::vector<AlphaArgs> al;
    std::vector<ControlArgs> ct;
    std::vector<ShiftArgs<T>> sh;
    std::vector<int32_t> omu{0}, oup{0}, oblk{0}, osh{0};
    for (SV* p : sv) {
      auto& S = p->S;
      auto& h = p->h;
      require(h.stream == st && h.nf == nf && S.g.variant == variant && S.kch == kch,
              "batched regions need one stream, one nf, one tile shape and one shift chunk");
      full = full && p->full_tiles(variant);
      cT* b0 = S.r0.template as<cT>();
      cT* b1 = S.r1.template as<cT>();
      ColState* cols = S.cols.template as<ColState>();
      int32_t* act = S.blk_active.template as<int32_t>();
      double2* part0 = S.part0.template as<double2>();
      double* part1 = S.part1.template as<double>();
      double2* partm = S.partm.template as<double2>();
      const StencilGrid gm = p->mu_grid();
      StencilArgs<T> m = p->stencil_args(MODE_MU, gm, S.nb, cols, act, partm, nullptr,
                                         S.dc.template as<cT>(), S.qa.template as<double2>());
      // x, p update of iteration n inside the mu launch of iteration n + 2
      m.shift = p->shift_args(SV::tile_cfg(h.nf == 4 ? variant : 1).nt, kch);
      m.nshift_wg = (m.shift.gx * m.shift.gy * S.nb + 7) / 8 * 8;
      StencilArgs<T> u = p->stencil_args(MODE_UPDATE, S.g, S.nb, cols, act, part0, part1,
                                         S.dc.template as<cT>(), nullptr);
      u.cache_mode = S.cache_mode;
      for (StencilArgs<T>* q : {&m, &u}) {
        q->pingpong = 1;
        q->bufs[0] = to_g(b0);
        q->bufs[1] = to_g(b1);
      }
      mu.push_back(m);
      omu.push_back(omu.back() + SV::stencil_wgs(m, gm));
      up.push_back(u);
      oup.push_back(oup.back() + SV::stencil_wgs(u, S.g));
      AlphaArgs aa{};
      aa.part = to_g(partm);
      aa.nwg = gm.nwg;
      aa.qa = to_g(S.qa.template as<double2>());
      aa.n_atoms = h.n_atoms;
      aa.cols = to_g(cols);
      aa.blk_active = to_g(act);
      al.push_back(aa);
      oblk.push_back(oblk.back() + S.nb);
      ControlArgs ca{};
      ca.part_rho = to_g(part0);
      ca.part_nu = to_g(part1);
      ca.nwg = S.nwg;
      ca.cols = to_g(cols);
      ca.sh = to_g(S.sh.template as<ShiftState>());
      ca.coef = to_g(S.coef.template as<ShiftCoef>());
      ca.z = to_g(S.z.template as<double2>());
      ca.K = S.K;
      ca.list = to_g(S.list.template as<int32_t>());
      ca.cnt = to_g(S.cnt.template as<int32_t>());
      ca.k5cnt = to_g(S.k5cnt.template as<int32_t>());
      ca.pim = to_g(S.pim.template as<double>());
      ca.act = to_g(S.act.template as<unsigned char>());
      ca.blk_active = to_g(act);
      ca.blk_iter = to_g(S.blk_iter.template as<int32_t>());
      ca.nb = S.nb;
      ca.tol = o.tol;
      ca.max_iter = o.max_iter;
      ca.seed_switch = o.seed_switch;
      ca.stall = SV::DBL ? 0 : kStallWindow;
      ca.floor_est = SV::DBL ? 0.0 : kMixedFloor;
      ct.push_back(ca);
      const ShiftArgs<T> sa = p->shift_args(WG, kch);
      sh.push_back(sa);
      const int64_t nsh = (int64_t)osh.back() + (int64_t)sa.gx * sa.gy * S.nb;
      require(nsh < (int64_t)1 << 31, "shift update grid too large");
      osh.push_back((int32_t)nsh);
      ctl_lds = std::max(ctl_lds, SV::control_lds(S.K));
    }
    upload(t_mu, mu, st);
    upload(t_upd, up, st);
    upload(t_alpha, al, st);
    upload(t_ctl, ct, st);
    upload(t_shift, sh, st);
    upload(o_mu, omu, st);
    upload(o_upd, oup, st);
    upload(o_blk, oblk, st);
    upload(o_shift, osh, st);
    g_mu = omu.back();
    g_upd = oup.back();
    g_blk = oblk.back();
    g_shift = osh.back();
    HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_control<B>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)ctl_lds));
  }

  int n() const { return (int)sv.size(); }

  // ev: null, or 2*SCOCG_K_FAMILIES events recorded around the launches of this
  // iteration; timing mode 1 records every family, mode 2 only the r_{n+1} pass
  void mark(hipEvent_t* ev, int fam, int end) {
    if (!ev || (timing_mode == 2 && fam != SCOCG_K_UPDATE)) return;
    HIPCHK(hipEventRecord(ev[2 * fam + end], st));
  }

  // Iteration s2 of a poll chunk of `poll` iterations (poll is a multiple of 6, so s2
  // mod 6 is the absolute iteration n mod 6): the mu launch of n also runs the control
  // step of n - 1 (except at the start of a chunk, whose previous control step ended
  // the last chunk) and the x, p update of n - 2; the chunk's last iteration runs its
  // control step alone, so that the host poll after the chunk sees it.
  void one_iteration(int s2, int poll, hipEvent_t* ev) {
    const int par = s2 & 1, n6 = s2 % 6;
    typename SV::CtlIn ci;
    if (s2 > 0) {
      ci.regs = t_ctl.as<ControlArgs>();
      ci.off = o_blk.as<int32_t>();
      ci.n = g_blk;
      ci.n6 = n6;
    }
    mark(ev, SCOCG_K_MU, 0);
    SV::template launch_table<MODE_MU>(st, nf, variant, full, t_mu.as<StencilArgs<T>>(),
                                       o_mu.as<int32_t>(), n(), g_mu, par, ci);
    mark(ev, SCOCG_K_MU, 1);
    mark(ev, SCOCG_K_ALPHA, 0);
    hipLaunchKernelGGL((k_alpha<B>), dim3(g_blk), dim3(WG), 0, st, t_alpha.as<AlphaArgs>(),
                       o_blk.as<int32_t>(), n(), par);
    KCHK();
    mark(ev, SCOCG_K_ALPHA, 1);
    mark(ev, SCOCG_K_UPDATE, 0);
    SV::template launch_table<MODE_UPDATE>(st, nf, variant, full, t_upd.as<StencilArgs<T>>(),
                                           o_upd.as<int32_t>(), n(), g_upd, par);
    mark(ev, SCOCG_K_UPDATE, 1);
    if (s2 == poll - 1) {
      mark(ev, SCOCG_K_CONTROL, 0);
      hipLaunchKernelGGL((k_control<B>), dim3(g_blk), dim3(CT), ctl_lds, st,
                         t_ctl.as<ControlArgs>(), o_blk.as<int32_t>(), n(), par, n6 % 3);
      KCHK();
      mark(ev, SCOCG_K_CONTROL, 1);
    }
  }

  // x, p update of iteration m (parity m mod 2, list m mod 3) outside the mu launches
  void flush_shift(int par, int lsel) {
    hipLaunchKernelGGL((k_shift<T, B>), dim3(g_shift), dim3(WG), 0, st,
                       t_shift.as<ShiftArgs<T>>(), o_shift.as<int32_t>(), n(), par, lsel);
    KCHK();
  }

  // Runs until every region's blocks are inactive (or the iteration cap).  With
  // t0 (an event recorded on the stream before the solve) and region_ms, the device
  // time from t0 to the poll at which each region finished is stored.
  int64_t iterate(const scocg_solve_opts& o, double* kms, int64_t* kcount, hipEvent_t t0,
                  double* region_ms) {
    int poll = o.poll_every > 0 ? o.poll_every : 16;
    // a multiple of 6: the buffer parity (2) and the list index (3) repeat per chunk,
    // so one captured chunk serves every chunk
    poll = (poll + 5) / 6 * 6;
    int64_t it = 0;
    Graph graph;
    // timing: one event pair per kernel family per iteration of a poll chunk
    timing_mode = o.timing;
    std::vector<Event> evs;
    if (o.timing) evs.resize((size_t)poll * 2 * SCOCG_K_FAMILIES);
    std::vector<hipEvent_t> evh;
    for (const auto& e : evs) evh.push_back(e);
    std::unique_ptr<Event> evp;
    if (t0 && region_ms) evp.reset(new Event());
    std::vector<char> done(sv.size(), 0);
    auto ev_of = [&](int s2) { return o.timing ? &evh[(size_t)s2 * 2 * SCOCG_K_FAMILIES] : nullptr; };
    // events recorded during capture cannot be read back after a replay on this
    // runtime (and an external event-record node, hipEventRecordWithFlags with
    // hipEventRecordExternal, is refused during capture): timing runs use direct
    // launches
    const bool use_graph = o.use_graph && !o.timing;
    while (true) {
      if (use_graph) {
        if (!graph.x) {
          HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
          try {
            for (int s2 = 0; s2 < poll; ++s2) one_iteration(s2, poll, ev_of(s2));
          } catch (...) {
            // leave the stream usable: end the capture and drop the partial graph
            hipGraph_t partial = nullptr;
            (void)hipStreamEndCapture(st, &partial);
            if (partial) (void)hipGraphDestroy(partial);
            throw;
          }
          HIPCHK(hipStreamEndCapture(st, &graph.g));
          HIPCHK(hipGraphInstantiate(&graph.x, graph.g, nullptr, nullptr, 0));
        }
        HIPCHK(hipGraphLaunch(graph.x, st));
      } else {
        for (int s2 = 0; s2 < poll; ++s2) one_iteration(s2, poll, ev_of(s2));
      }
      it += poll;
      if (evp) HIPCHK(hipEventRecord(*evp, st));
      for (SV* p : sv)
        HIPCHK(hipMemcpyAsync(p->S.h_flags, p->S.blk_active.p, p->S.nb * sizeof(int32_t),
                              hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (o.timing) {
        for (int s2 = 0; s2 < poll; ++s2)
          for (int f = 0; f < SCOCG_K_FAMILIES; ++f) {
            // the projector contraction, the x, p update and (but at the end of a
            // chunk) the control step run inside the MU launch
            if (f == SCOCG_K_PROJ || f == SCOCG_K_SHIFT) continue;
            if (f == SCOCG_K_CONTROL && s2 != poll - 1) continue;
            if (o.timing == 2 && f != SCOCG_K_UPDATE) continue;
            float t = 0.f;
            hipEvent_t* e = ev_of(s2);
            HIPCHK(hipEventElapsedTime(&t, e[2 * f], e[2 * f + 1]));
            kms[f] += t;
            kcount[f] += 1;
          }
      }
      int any_all = 0;
      for (size_t r = 0; r < sv.size(); ++r) {
        int any = 0;
        for (int b = 0; b < sv[r]->S.nb; ++b) any |= sv[r]->S.h_flags[b];
        if (!any && !done[r]) {
          done[r] = 1;
          if (evp) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, t0, *evp));
            region_ms[r] = ms;
          }
        }
        any_all |= any;
      }
      if (trace_level() >= 2 && it % 2048 == 0) {
        int left = 0;
        for (char d : done) left += !d;
        fprintf(stderr, "[scocg] %lld seed iterations, %d of %d regions active\n", (long long)it,
                left, (int)sv.size());
      }
      if (!any_all || it >= o.max_iter + poll) break;
    }
    // the x, p updates of the last two iterations (it is a multiple of 6): iteration
    // it - 2 has parity 0 and list 1, it - 1 parity 1 and list 2
    flush_shift(0, 1);
    flush_shift(1, 2);
    return it;
  }
};

template <typename T, int B>
int64_t Solver<T, B>::iterate(const scocg_solve_opts& o, double* kms, int64_t* kcount) {
  Batch<T, B> bt({this}, o);
  return bt.iterate(o, kms, kcount, nullptr, nullptr);
}

// ---- streaming bandwidth probe (scocg_stream_probe): the access mixes of the stencil
// passes without their arithmetic.  Each thread moves U 16-byte vectors per step of a
// grid-stride loop over n vectors; loads of one step are issued before its stores.
//   NR = 1: c = a            (a copy: one read, one write)
//   NR = 2: c = a + b        (the r_{n+1} pass: two reads, one write)
//   NR = 0: s += a           (the mu pass: reads only; one value per workgroup written)
template <int NR, bool NT, int U>
__global__ __launch_bounds__(256) void k_stream(const double2* __restrict__ a,
                                                const double2* __restrict__ b,
                                                double2* __restrict__ c, int64_t n,
                                                double* __restrict__ sink) {
  const int64_t stride = (int64_t)gridDim.x * 256 * U;
  double2 acc = mk(0, 0);
  for (int64_t i0 = (int64_t)blockIdx.x * 256 * U + threadIdx.x; i0 < n; i0 += stride) {
    double2 va[U], vb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + (int64_t)u * 256;
      if (i < n) {
        va[u] = NT ? ld_stream(a + i) : a[i];
        if (NR == 2) vb[u] = NT ? ld_stream(b + i) : b[i];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + (int64_t)u * 256;
      if (i >= n) continue;
      if (NR == 0) {
        acc = cadd(acc, va[u]);
      } else {
        const double2 v = NR == 2 ? cadd(va[u], vb[u]) : va[u];
        if (NT) st_stream(c + i, v);
        else c[i] = v;
      }
    }
  }
  if (NR == 0) {
    __shared__ double sh[256];
    sh[threadIdx.x] = acc.x + acc.y;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) sink[blockIdx.x] = sh[0];
  }
}

// ---- operator apply y = H x (scocg_apply_h and its allocation-free variant)

// one-entry argument table of a stencil launch (and its workgroup offsets {0, grid}),
// written on the stream instead of copied from the host
template <typename T>
__global__ void k_put_table(StencilArgs<T> a, StencilArgs<T>* __restrict__ tab,
                            int32_t* __restrict__ off, int grid) {
  if (threadIdx.x == 0) {
    *tab = a;
    off[0] = 0;
    off[1] = grid;
  }
}


// Device workspace of one apply: x scattered into column 0 of a padded column block,
// the stencil output block, the projector coefficients D_a P_a^T x, and the one-entry
// argument table of the stencil launch (written by a kernel, not uploaded).  Offsets
// are 256-byte aligned inside one region of apply_ws_bytes() bytes.
template <typename T, int B>
struct ApplyWs {
  using cT = typename cplx_of<T>::type;
  size_t o_tab = 0, o_off = 0, o_dc = 0, o_pc = 0, o_blk = 0, o_out = 0, bytes = 0;
  bool pc = false;  // per-entry projector products (the matrix-core application)
  explicit ApplyWs(const scocg_ctx& h) {
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t blk = (((size_t)h.nz + 2 * h.nf) * h.nxy * B) * sizeof(cT);
    pc = std::is_same<T, float>::value && h.proj_mfma && h.n_atoms > 0;
    o_tab = 0;
    o_off = up(sizeof(StencilArgs<T>));
    o_dc = o_off + 256;
    o_pc = o_dc + up((size_t)std::max(h.n_atoms, 1) * 4 * B * sizeof(cT));
    o_blk = o_pc + (pc ? up((size_t)h.n_ent * B * sizeof(cT)) : 0);
    o_out = o_blk + up(blk);
    bytes = o_out + up(blk);
  }
};

template <typename T, int B>
void apply_h_run(scocg_ctx& h, const void* x, void* y, char* ws) {
  using cT = typename cplx_of<T>::type;
  const ApplyWs<T, B> L(h);
  auto* tab = reinterpret_cast<StencilArgs<T>*>(ws + L.o_tab);
  auto* off = reinterpret_cast<int32_t*>(ws + L.o_off);
  cT* dc = reinterpret_cast<cT*>(ws + L.o_dc);
  cT* blk = reinterpret_cast<cT*>(ws + L.o_blk);
  cT* out = reinterpret_cast<cT*>(ws + L.o_out);
  scocg_ctx::Solve tmp;  // no buffers: the solver object only plans and fills arguments
  Solver<T, B> sv(h, tmp);
  // every element of blk (padding planes and columns 1.. zero), of dc and of the
  // interior planes of out that the gather reads is written below: nothing needs clearing
  hipLaunchKernelGGL((k_scatter_col0<T, B>), dim3(nblocks(sv.bstride(), WG)), dim3(WG), 0,
                     h.stream, static_cast<const double2*>(x), blk, sv.bstride(), h.N,
                     sv.pad_points());
  KCHK();
  sv.launch_proj(blk, 1, dc, nullptr);
  const auto g = sv.plan(1, 0, 0);
  StencilArgs<T> a = sv.stencil_args(MODE_APPLY, g, 1, nullptr, nullptr, nullptr, nullptr, dc,
                                     nullptr);
  a.r = to_g(static_cast<const cT*>(blk));
  a.io = to_g(out);
  if constexpr (std::is_same<T, float>::value) {
    if (L.pc) {  // complex64: the application P_a (D_a C_a) on matrix cores as well
      float2* pc = reinterpret_cast<float2*>(ws + L.o_pc);
      hipLaunchKernelGGL((k_proj_apply_mfma<WG>), dim3(h.n_atoms, 1), dim3(WG), 0, h.stream,
                         sv.proj_args(dc, nullptr), (int)h.n_ent, pc);
      KCHK();
      a.pcv = to_g(static_cast<const float2*>(pc));
      a.pent = to_g(h.pent.as<int32_t>());
      a.n_ent = (int)h.n_ent;
    }
  }
  const int grid = Solver<T, B>::stencil_wgs(a, g);
  hipLaunchKernelGGL((k_put_table<T>), dim3(1), dim3(1), 0, h.stream, a, tab, off, grid);
  KCHK();
  Solver<T, B>::template launch_table<MODE_APPLY>(h.stream, h.nf, g.variant,
                                                  sv.full_tiles(g.variant), tab, off, 1, grid, 0);
  hipLaunchKernelGGL((k_gather_col0<T, B>), dim3(nblocks(h.N, WG)), dim3(WG), 0, h.stream, out,
                     static_cast<double2*>(y), h.N, sv.pad_points());
  KCHK();
  HIPCHK(hipStreamSynchronize(h.stream));
}

template <typename T, int B>
void apply_h_impl(scocg_ctx& h, const void* x, void* y) {
  DevBuf ws;
  ws.alloc(ApplyWs<T, B>(h).bytes);
  apply_h_run<T, B>(h, x, y, ws.as<char>());
}

bool all_finite(const double* p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

template <typename F>
int guarded(F&& f) {
  try {
    g_err.clear();
    return f();
  } catch (const Error& e) {
    g_err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return SCOCG_ENOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return SCOCG_EHIP;
  }
}


// [p, p + bytes) must lie inside one device allocation of `device`: a host or
// foreign pointer, or a buffer too small for the shape, is an argument error
// here rather than a memory fault inside a kernel.
void require_device_range(const void* p, size_t bytes, int device, const char* name) {
  require(p != nullptr, std::string(name) + " is NULL");
  hipPointerAttribute_t at{};
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    require(false, std::string(name) + " is not device memory");
  }
  require(at.type == hipMemoryTypeDevice && at.device == device,
          std::string(name) + " is not device memory of the handle's device");
  void* base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) != hipSuccess) {
    (void)hipGetLastError();
    require(false, std::string(name) + ": allocation range unknown");
  }
  require(static_cast<const char*>(p) + bytes <= static_cast<const char*>(base) + size,
          std::string(name) + " is smaller than the shape requires");
}

// Open-boundary matching on the device (see obm_kernels.hpp) for K energies,
// boundary blocks of M rows each and L extra rows; D = 2M + L, n = 2M.
//   g [K][D][D], sig_l, sig_r [K][M][M] inputs; gt [K][D][D] output (device).
//   T [K] complex transmission, dos [K] (device scratch, copied out by the caller).
// Returns the number of energies whose elimination met a zero pivot.
int obm_run(scocg_ctx& h, int K, int M, int L, const double2* g, const double2* sig_l,
            const double2* sig_r, double2* gt, std::vector<double2>& T_host,
            std::vector<double>& dos_host, double* phase_ms) {
  hipStream_t st = h.stream;
  // optional device timing: an event pair around every launch of each phase
  // (0 setup products, 1 panels, 2 panel updates, 3 outputs, T and DOS)
  std::vector<std::unique_ptr<Event>> evs;
  std::vector<int> ev_phase;
  auto mark = [&](int phase) {
    if (!phase_ms) return;
    evs.emplace_back(new Event());
    HIPCHK(hipEventRecord(evs.back()->e, st));
    ev_phase.push_back(phase);
  };
  const int n = 2 * M, D = 2 * M + L, ncol = n + D;
  DevBuf W, f, piv, Vj, fail, P, GR, U, Q, T, dos, lists;
  W.alloc(sizeof(double2) * (size_t)K * n * ncol);
  Vj.alloc(sizeof(double2) * (size_t)K * obm::GJ_W * ncol);
  f.alloc(sizeof(double2) * (size_t)K * n * obm::GJ_W);
  piv.alloc(sizeof(double2) * (size_t)K * obm::GJ_W);
  fail.alloc(sizeof(int32_t) * K);
  GR.alloc(sizeof(double2) * (size_t)K * M * M);
  U.alloc(sizeof(double2) * (size_t)K * M * M);
  Q.alloc(sizeof(double2) * (size_t)K * M * M);
  T.alloc(sizeof(double2) * K);
  dos.alloc(sizeof(double) * K);
  if (L > 0) P.alloc(sizeof(double2) * (size_t)K * L * n);
  double2* Wp = W.as<double2>();
  const size_t Wstride = (size_t)n * ncol, gstride = (size_t)D * D, sstride = (size_t)M * M;
  const size_t Pstride = (size_t)L * n;

  // pointer lists of every batched product, uploaded once
  std::vector<obm::GemmPtrs> hl;
  const size_t o_build = hl.size();  // W(b_r, b_c) -= G(b_r, b_c) Sigma_c
  for (int k = 0; k < K; ++k)
    for (int c = 0; c < 2; ++c)
      for (int r = 0; r < 2; ++r)
        hl.push_back({g + k * gstride + (size_t)r * M + (size_t)D * c * M,
                      (c == 0 ? sig_l : sig_r) + k * sstride,
                      Wp + k * Wstride + (size_t)r * M + (size_t)n * c * M});
  const size_t o_p = hl.size();  // P(:, c-block) = G(l, b_c) Sigma_c
  if (L > 0)
    for (int k = 0; k < K; ++k)
      for (int c = 0; c < 2; ++c)
        hl.push_back({g + k * gstride + n + (size_t)D * c * M,
                      (c == 0 ? sig_l : sig_r) + k * sstride,
                      P.as<double2>() + k * Pstride + (size_t)L * c * M});
  const size_t o_px = hl.size();  // G_T(l, :) += P X
  if (L > 0)
    for (int k = 0; k < K; ++k)
      hl.push_back({P.as<double2>() + k * Pstride, Wp + k * Wstride + (size_t)n * n,
                    gt + k * gstride + n});
  const size_t o_u = hl.size();  // U = Gamma_R Y, Y = X(right rows, left columns)
  for (int k = 0; k < K; ++k)
    hl.push_back({GR.as<double2>() + k * sstride, Wp + k * Wstride + (size_t)n * n + M,
                  U.as<double2>() + k * sstride});
  const size_t o_q = hl.size();  // Q = Y^H U
  for (int k = 0; k < K; ++k)
    hl.push_back({Wp + k * Wstride + (size_t)n * n + M, U.as<double2>() + k * sstride,
                  Q.as<double2>() + k * sstride});
  lists.alloc(sizeof(obm::GemmPtrs) * hl.size());
  HIPCHK(hipMemcpyAsync(lists.p, hl.data(), lists.bytes, hipMemcpyHostToDevice, st));
  const obm::GemmPtrs* dl = lists.as<obm::GemmPtrs>();
  auto gemm = [&](size_t off, int batch, bool conj_a, int m, int nn, int kd, int lda, int ldb,
                  int ldc, double2 alpha, double2 beta, int beta_zero) {
    dim3 grid(nblocks(m, obm::GT), nblocks(nn, obm::GT), batch);
    if (conj_a)
      hipLaunchKernelGGL(obm::k_zgemm<true>, grid, dim3(256), 0, st, dl + off, m, nn, kd, lda,
                         ldb, ldc, alpha, beta, beta_zero);
    else
      hipLaunchKernelGGL(obm::k_zgemm<false>, grid, dim3(256), 0, st, dl + off, m, nn, kd, lda,
                         ldb, ldc, alpha, beta, beta_zero);
    KCHK();
  };
  const double2 one = {1.0, 0.0}, mone = {-1.0, 0.0}, zero = {0.0, 0.0};

  // 1. W = [I | G(b, :)], then W(:, 0:n) -= G_bb Sigma_b
  HIPCHK(hipMemsetAsync(fail.p, 0, fail.bytes, st));
  mark(0);
  hipLaunchKernelGGL(obm::k_obm_init, dim3(ncol, nblocks(n, 256), K), dim3(256), 0, st, g, Wp,
                     n, D);
  KCHK();
  gemm(o_build, 4 * K, false, M, M, M, D, M, n, mone, one, 0);
  mark(0);
  // 2. Gauss-Jordan by panels: W(:, n:) becomes G_T(b, :)
  for (int j0 = 0; j0 < n; j0 += obm::GJ_W) {
    const int w = std::min(obm::GJ_W, n - j0);
    mark(1);
    if (n <= 1024)  // each thread keeps at most two rows per pivot step
      hipLaunchKernelGGL(obm::k_gj_panel<512>, dim3(K), dim3(512), 0, st, Wp, f.as<double2>(),
                         piv.as<double2>(), Vj.as<double2>(), fail.as<int32_t>(), n, ncol, j0, w);
    else
      hipLaunchKernelGGL(obm::k_gj_panel<1024>, dim3(K), dim3(1024), 0, st, Wp, f.as<double2>(),
                         piv.as<double2>(), Vj.as<double2>(), fail.as<int32_t>(), n, ncol, j0, w);
    KCHK();
    const int cols = ncol - j0 - w;  // > 0: the RHS columns always follow
    mark(1);
    mark(2);
    hipLaunchKernelGGL(obm::k_gj_sweep, dim3(nblocks(cols, 64), K), dim3(64), 0, st,
                       Vj.as<double2>(), f.as<double2>(), piv.as<double2>(), fail.as<int32_t>(),
                       n, ncol, j0, w);
    KCHK();
    hipLaunchKernelGGL(obm::k_gj_update, dim3(nblocks(cols, obm::GJ_T), nblocks(n, obm::GJ_T), K),
                       dim3(256), 0, st, Wp, f.as<double2>(), Vj.as<double2>(),
                       fail.as<int32_t>(), n, ncol, j0, w);
    KCHK();
    mark(2);
  }
  // 3. output rows: boundary rows from X, extra rows G(l, :) + G(l, b) Sigma_b X
  mark(3);
  hipLaunchKernelGGL(obm::k_obm_out, dim3(D, nblocks(D, 256), K), dim3(256), 0, st, Wp, g, gt,
                     fail.as<int32_t>(), n, D);
  KCHK();
  if (L > 0) {
    gemm(o_p, 2 * K, false, L, M, M, D, M, L, one, zero, 1);
    gemm(o_px, K, false, L, D, n, L, n, D, one, one, 0);
  }
  // 4. T = Tr[Gamma_L Y^H Gamma_R Y]
  hipLaunchKernelGGL(obm::k_gamma, dim3(M, nblocks(M, 256), K), dim3(256), 0, st, sig_r,
                     GR.as<double2>(), M);
  KCHK();
  gemm(o_u, K, false, M, M, M, M, n, M, one, zero, 1);
  gemm(o_q, K, true, M, M, M, n, M, M, one, zero, 1);
  hipLaunchKernelGGL(obm::k_trace_gamma, dim3(K), dim3(256), 0, st, sig_l, Q.as<double2>(),
                     T.as<double2>(), fail.as<int32_t>(), M);
  KCHK();
  hipLaunchKernelGGL(obm::k_dos, dim3(K), dim3(256), 0, st, gt, dos.as<double>(),
                     fail.as<int32_t>(), n, D, L);
  KCHK();
  mark(3);
  std::vector<int32_t> fl(K);
  T_host.resize(K);
  dos_host.resize(K);
  HIPCHK(hipMemcpyAsync(T_host.data(), T.p, T.bytes, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(dos_host.data(), dos.p, dos.bytes, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(fl.data(), fail.p, fail.bytes, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));  // every workspace buffer is freed on return
  if (phase_ms) {
    for (int q = 0; q < 4; ++q) phase_ms[q] = 0.0;
    for (size_t e = 0; e + 1 < evs.size(); e += 2)
      phase_ms[ev_phase[e]] += elapsed_ms(*evs[e], *evs[e + 1]);
  }
  int nfail = 0;
  for (int v : fl) nfail += v != 0;
  return nfail;
}

}  // namespace

// ------------------------------------------------------------------------------------ C ABI
namespace {

// argument checks shared by scocg_solve and scocg_batch_solve
void check_problem(const scocg_ctx* h, int32_t K, const double* z, int32_t R,
                   const int64_t* rhs_idx, int32_t nS, const int64_t* s_idx, bool full) {
  require(h != nullptr, "handle is NULL");
  require(K >= 1 && z != nullptr, "need K >= 1 energies");
  require(R >= 1 && rhs_idx != nullptr, "need R >= 1 right-hand sides");
  for (int k = 0; k < K; ++k) {
    require(std::isfinite(z[2 * k]) && std::isfinite(z[2 * k + 1]), "non-finite energy");
    require(z[2 * k + 1] > 0.0, "every energy needs Im z > 0");
  }
  for (int j = 0; j < R; ++j) require(rhs_idx[j] >= 0 && rhs_idx[j] < h->N, "rhs_idx out of range");
  if (!full) {
    if (s_idx) {
      require(nS >= 1, "nS must be >= 1 with s_idx");
      for (int i = 0; i < nS; ++i) require(s_idx[i] >= 0 && s_idx[i] < h->N, "s_idx out of range");
    } else {
      require(nS == 0, "nS > 0 needs s_idx");
    }
  }
}

scocg_solve_opts check_opts(const scocg_solve_opts* opts) {
  scocg_solve_opts o{};
  if (opts) o = *opts;
  if (!(o.tol > 0.0)) o.tol = 1e-10;
  require(std::isfinite(o.tol), "non-finite tol");
  if (o.max_iter <= 0) o.max_iter = 100000;
  require(o.timing >= 0 && o.timing <= 2, "timing must be 0, 1 or 2");
  require(o.tile >= SCOCG_AUTO && o.tile <= 4, "tile must be SCOCG_AUTO or 0..4");
  require(o.zchunk >= SCOCG_AUTO, "zchunk must be SCOCG_AUTO or >= 0");
  require(o.zchunk_mu >= SCOCG_AUTO, "zchunk_mu must be SCOCG_AUTO or >= 0");
  require(o.cache_mode >= SCOCG_AUTO && o.cache_mode <= 2,
          "cache_mode must be SCOCG_AUTO, 0, 1 or 2");
  require(o.shift_chunk == SCOCG_AUTO || o.shift_chunk == 0 || o.shift_chunk == 1 ||
              o.shift_chunk == 4 || o.shift_chunk == 16,
          "shift_chunk must be SCOCG_AUTO, 0, 1, 4 or 16");
  require(o.conventional == 0 || o.conventional == 1, "conventional must be 0 or 1");
  require(o.aux_seed == 0 || o.aux_seed == 1, "aux_seed must be 0 or 1");
  require(o.symmetric == 0 || o.symmetric == 1, "symmetric must be 0 or 1");
  require(!o.symmetric || (o.full == 0 && o.conventional == 0),
          "symmetric needs projected storage and the shifted solve");
  if (o.aux_seed) {
    require(std::isfinite(o.seed_z[0]) && std::isfinite(o.seed_z[1]) && o.seed_z[1] > 0.0,
            "seed_z must be finite with Im > 0");
    require(o.conventional == 0, "aux_seed does not apply to the conventional sweep");
  }
  return o;
}

// All regions: prepare, one shared iteration loop (one launch per kernel family per
// iteration), then per region the FP64 checks / refinement and the report.
// Autotuning of a batch: one tile shape and one shift chunk serve every region (they
// select the kernel instances of the shared launches); each region keeps the z-chunk
// its own plan gives for that tile (zchunk = SCOCG_AUTO), or the explicit one.  Each
// candidate is timed as 16 iterations of the whole batch from its initial state; the
// winner is kept in every region's state.  Returns the device ms of the trials.
template <typename T, int B>
double tune_batch(std::vector<Solver<T, B>*>& ptr, const scocg_solve_opts& o, bool want_tile,
                  bool want_kch, bool want_cache) {
  constexpr int kIters = 16;
  hipStream_t st = ptr[0]->h.stream;
  scocg_solve_opts ot = o;
  ot.max_iter = kIters;
  ot.timing = 0;
  ot.use_graph = 0;
  ot.poll_every = kIters;
  const int zc_fixed = o.zchunk > 0 ? o.zchunk : 0;
  auto trial = [&]() {
    for (auto* p : ptr)
      p->init_unit(p->zk.template as<double2>(), p->seed0,
                   p->conv ? p->zk.template as<double2>() : nullptr);
    Event a, b;
    HIPCHK(hipEventRecord(a, st));
    double km[SCOCG_K_FAMILIES] = {0};
    int64_t kc[SCOCG_K_FAMILIES] = {0};
    Batch<T, B> bt(ptr, ot);
    bt.iterate(ot, km, kc, nullptr, nullptr);
    HIPCHK(hipEventRecord(b, st));
    return elapsed_ms(a, b);
  };
  auto set_tile = [&](int v) {
    for (auto* p : ptr) p->set_grid(p->plan(p->S.nb, v, zc_fixed));
  };
  Event t0, t1;
  HIPCHK(hipEventRecord(t0, st));
  if (want_tile && ptr[0]->h.nf == 4) {
    double best = INFINITY;
    int bv = ptr[0]->S.g.variant;
    for (int v : {1, 2, 3, 4}) {
      set_tile(v);
      const double ms = trial();
      if (trace_on()) fprintf(stderr, "[scocg] batch tune tile %d: %.3f ms\n", v, ms);
      if (ms < best) {
        best = ms;
        bv = v;
      }
    }
    set_tile(bv);
  }
  if (want_kch) {
    double best = INFINITY;
    int bk = ptr[0]->S.kch;
    for (int kch : {1, 4, 16}) {
      for (auto* p : ptr) p->S.kch = kch;
      const double ms = trial();
      if (trace_on()) fprintf(stderr, "[scocg] batch tune shift chunk %d: %.3f ms\n", kch, ms);
      if (ms < best) {
        best = ms;
        bk = kch;
      }
    }
    for (auto* p : ptr) p->S.kch = bk;
  }
  if (want_cache) {
    double best = INFINITY;
    int bm = 0;
    for (int m : {0, 1, 2}) {
      for (auto* p : ptr) p->S.cache_mode = m;
      const double ms = trial();
      if (trace_on()) fprintf(stderr, "[scocg] batch tune cache mode %d: %.3f ms\n", m, ms);
      if (ms < best) {
        best = ms;
        bm = m;
      }
    }
    for (auto* p : ptr) p->S.cache_mode = bm;
  }
  HIPCHK(hipEventRecord(t1, st));
  return elapsed_ms(t0, t1);
}

template <typename T, int B>
int run_batch(int n, const scocg_handle* hs, const scocg_problem* pr, scocg_solve_opts o,
              scocg_report* reps, double* region_ms) {
  // SCOCG_AUTO: one tile shape and shift chunk for the whole batch, tuned on the batch
  // itself before the timed region; z-chunks stay per region (each region's plan)
  const bool auto_tile = o.tile == SCOCG_AUTO, auto_kch = o.shift_chunk == SCOCG_AUTO,
             auto_cache = o.cache_mode == SCOCG_AUTO;
  if (o.tile == SCOCG_AUTO) o.tile = 0;
  if (o.zchunk == SCOCG_AUTO) o.zchunk = 0;
  if (o.shift_chunk == SCOCG_AUTO) o.shift_chunk = 0;
  if (o.cache_mode == SCOCG_AUTO) o.cache_mode = 0;
  if (o.zchunk_mu == SCOCG_AUTO) o.zchunk_mu = 0;  // each region's mu pass follows its zchunk
  std::vector<std::unique_ptr<Solver<T, B>>> sv;
  std::vector<Solver<T, B>*> ptr;
  for (int i = 0; i < n; ++i) {
    hs[i]->last.reset(new scocg_ctx::Solve());
    sv.emplace_back(new Solver<T, B>(*hs[i], *hs[i]->last));
    scocg_solve_opts oi = o;
    if (oi.init_seed >= pr[i].K) oi.init_seed = -1;
    sv.back()->prepare(pr[i].K, pr[i].z, pr[i].R, pr[i].rhs_idx, pr[i].nS, pr[i].s_idx, oi);
    ptr.push_back(sv.back().get());
  }
  double tune_ms = 0.0;
  if (auto_tile || auto_kch || auto_cache)
    tune_ms = tune_batch<T, B>(ptr, o, auto_tile, auto_kch, auto_cache);
  hipStream_t st = hs[0]->stream;
  Event e0, e1;
  HIPCHK(hipEventRecord(e0, st));
  for (auto* p : ptr)
    p->init_unit(p->zk.template as<double2>(), p->seed0,
                 p->conv ? p->zk.template as<double2>() : nullptr);
  double kms[SCOCG_K_FAMILIES] = {0};
  int64_t kcount[SCOCG_K_FAMILIES] = {0};
  std::vector<double> done_ms(n, 0.0);
  int64_t it_main = 0;
  {
    Batch<T, B> bt(ptr, o);
    it_main = bt.iterate(o, kms, kcount, e0, done_ms.data());
  }
  std::vector<std::vector<double>> tres(n);
  std::vector<int64_t> refined(n, 0);
  for (int i = 0; i < n; ++i) {
    refined[i] = ptr[i]->post(o, it_main, tres[i]);
    // refinement, where it runs, extends the region's completion past the loop
    if (!tres[i].empty() && refined[i] > 0) {
      HIPCHK(hipEventRecord(e1, st));
      done_ms[i] = elapsed_ms(e0, e1);
    }
  }
  HIPCHK(hipEventRecord(e1, st));
  const float ms = elapsed_ms(e0, e1);
  int rc = SCOCG_OK;
  for (int i = 0; i < n; ++i) {
    const int r = ptr[i]->report(o, tres[i], refined[i], ms, kms, kcount, tune_ms,
                                 tune_ms > 0.0, reps ? &reps[i] : nullptr);
    if (r == SCOCG_BREAKDOWN || (r == SCOCG_NOT_ALL_CONVERGED && rc == SCOCG_OK)) rc = r;
    if (region_ms) region_ms[i] = done_ms[i];
  }
  return rc;
}

}  // namespace

extern "C" {

int scocg_create(const scocg_grid* g, const double* coef, const double* vloc, int32_t n_atoms,
                 const int64_t* atom_ptr, const int64_t* atom_idx, const double* atom_P,
                 const double* atom_D, int32_t precision, void* hip_stream, scocg_handle* out) {
  return guarded([&]() -> int {
    require(out != nullptr, "out is NULL");
    *out = nullptr;
    require(g != nullptr && coef != nullptr && vloc != nullptr, "grid, coef or vloc is NULL");
    require(g->nf >= 1 && g->nf <= 4, "nf must be 1..4");
    require(g->nx >= g->nf && g->ny >= g->nf && g->nz >= 1, "need nx, ny >= nf and nz >= 1");
    // one padded column block ((nz + 2 nf) planes x 128 bytes per point) must be
    // addressable with 32-bit byte offsets
    require(g->nx * g->ny <= (1 << 30) &&
                (g->nz + 2 * g->nf) * g->nx * g->ny * 128 < ((int64_t)1 << 32),
            "grid too large for 32-bit offsets within a column block");
    require(g->n_proj >= 0 && g->n_proj <= 4, "n_proj must be 0..4");
    require(precision == SCOCG_FP64 || precision == SCOCG_MIXED, "unknown precision");
    require(n_atoms >= 0, "n_atoms < 0");
    auto h = std::make_unique<scocg_ctx>();
    h->nx = (int)g->nx;
    h->ny = (int)g->ny;
    h->nz = (int)g->nz;
    h->nxy = h->nx * h->ny;
    h->N = (int64_t)h->nxy * h->nz;
    h->nf = g->nf;
    h->n_proj = g->n_proj;
    h->precision = precision;
    // SCOCG_PROJ=mfma puts the complex64 projector contraction (and the application in
    // scocg_apply_h) on FP32 matrix cores; the vector-ALU paths are the default (faster
    // for this 4-channel contraction, measured)
    {
      const char* pe = getenv("SCOCG_PROJ");
      h->proj_mfma = precision == SCOCG_MIXED && pe && std::string(pe) == "mfma";
    }
    HIPCHK(hipGetDevice(&h->device));
    init_scratch(h->device);
    {
      hipDeviceProp_t prop;
      HIPCHK(hipGetDeviceProperties(&prop, h->device));
      h->arch = prop.gcnArchName;
      const size_t colon = h->arch.find(':');
      if (colon != std::string::npos) h->arch.resize(colon);
    }
    h->stream = static_cast<hipStream_t>(hip_stream);
    if (!h->stream) {  // a private stream, so that solves can be graph-captured
      HIPCHK(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
      h->own_stream = true;
    }
    require(all_finite(coef, 3 * (g->nf + 1)), "non-finite stencil coefficient");
    require(all_finite(vloc, h->N), "non-finite local potential");
    h->coef.assign(coef, coef + 3 * (g->nf + 1));
    if (n_atoms > 0) {
      require(g->n_proj >= 1, "atoms given but n_proj = 0");
      require(atom_ptr && atom_idx && atom_P && atom_D, "atom arrays are NULL");
      require(atom_ptr[0] == 0, "atom_ptr[0] != 0");
      for (int a = 0; a < n_atoms; ++a) {
        require(atom_ptr[a + 1] >= atom_ptr[a], "atom_ptr decreasing");
        std::vector<int64_t> idx(atom_idx + atom_ptr[a], atom_idx + atom_ptr[a + 1]);
        for (int64_t v : idx) require(v >= 0 && v < h->N, "atom_idx out of range");
        std::sort(idx.begin(), idx.end());
        require(std::adjacent_find(idx.begin(), idx.end()) == idx.end(),
                "grid index repeated within one atom");
      }
      require(atom_ptr[n_atoms] < ((int64_t)1 << 31), "too many projector entries");
      require(all_finite(atom_P, atom_ptr[n_atoms] * g->n_proj), "non-finite projector value");
      require(all_finite(atom_D, (int64_t)n_atoms * g->n_proj), "non-finite projector energy");
    }
    h->n_atoms = n_atoms;
    if (precision == SCOCG_FP64) {
      upload_operator<double>(*h, vloc, atom_ptr, atom_idx, atom_P, atom_D);
    } else {
      upload_operator<float>(*h, vloc, atom_ptr, atom_idx, atom_P, atom_D);
      upload_operator64(*h, vloc, atom_ptr, atom_idx, atom_P, atom_D);
    }
    *out = h.release();
    return SCOCG_OK;
  });
}


int scocg_solve(scocg_handle h, int32_t K, const double* z, int32_t R, const int64_t* rhs_idx,
                int32_t nS, const int64_t* s_idx, const scocg_solve_opts* opts,
                scocg_report* rep) {
  return guarded([&]() -> int {
    const scocg_solve_opts o = check_opts(opts);
    check_problem(h, K, z, R, rhs_idx, nS, s_idx, o.full != 0);
    require(!o.symmetric || s_idx == nullptr, "symmetric needs S = the RHS set (s_idx NULL)");
    require(o.init_seed >= -1 && o.init_seed < K, "init_seed out of range");
    HIPCHK(hipSetDevice(h->device));
    h->last.reset(new scocg_ctx::Solve());
    if (h->precision == SCOCG_FP64) {
      Solver<double, 8> sv(*h, *h->last);
      return sv.run(K, z, R, rhs_idx, nS, s_idx, o, rep);
    }
    Solver<float, 16> sv(*h, *h->last);
    return sv.run(K, z, R, rhs_idx, nS, s_idx, o, rep);
  });
}

int scocg_batch_solve(int32_t n, const scocg_handle* hs, const scocg_problem* probs,
                      const scocg_solve_opts* opts, scocg_report* reps, double* region_ms) {
  return guarded([&]() -> int {
    require(n >= 1 && hs != nullptr && probs != nullptr, "need n >= 1 handles and problems");
    const scocg_solve_opts o = check_opts(opts);
    require(o.init_seed == -1, "init_seed must be -1 (each region's middle energy) in a batch");
    require(o.aux_seed == 0, "aux_seed is not offered in a batch");
    for (int i = 0; i < n; ++i) {
      const scocg_problem& p = probs[i];
      check_problem(hs[i], p.K, p.z, p.R, p.rhs_idx, p.nS, p.s_idx, o.full != 0);
      require(!o.symmetric || p.s_idx == nullptr, "symmetric needs S = the RHS set (s_idx NULL)");
      require(hs[i]->device == hs[0]->device && hs[i]->stream == hs[0]->stream,
              "batched handles need one device and one stream");
      require(hs[i]->precision == hs[0]->precision && hs[i]->nf == hs[0]->nf,
              "batched handles need one precision and one nf");
      for (int j = 0; j < i; ++j) require(hs[j] != hs[i], "a handle appears twice in the batch");
    }
    HIPCHK(hipSetDevice(hs[0]->device));
    if (hs[0]->precision == SCOCG_FP64) return run_batch<double, 8>(n, hs, probs, o, reps, region_ms);
    return run_batch<float, 16>(n, hs, probs, o, reps, region_ms);
  });
}

int scocg_green_columns(scocg_handle h, void* dst, int32_t dtype, int32_t dst_is_device) {
  return guarded([&]() -> int {
    require(h != nullptr && dst != nullptr, "handle or dst is NULL");
    require(dtype == SCOCG_C128 || dtype == SCOCG_C64, "unknown dtype");
    if (!h->last || !h->last->ok) throw Error(SCOCG_ENOSOLVE, "no successful solve to copy");
    HIPCHK(hipSetDevice(h->device));
    auto& S = *h->last;
    // energy-major layout: the returned energies are the first Kout of the K gathered
    const int64_t tot_all = (int64_t)S.K * S.R * S.nS;
    const int64_t tot = (int64_t)S.Kout * S.R * S.nS;
    const size_t esz = dtype == SCOCG_C128 ? 16 : 8;
    DevBuf tmp;
    void* d = dst;
    if (dst_is_device) require_device_range(dst, (size_t)tot * esz, h->device, "dst");
    const bool staged = !dst_is_device || tot_all != tot;
    if (staged) {
      tmp.alloc(tot_all * esz);
      d = tmp.p;
    }
    const unsigned nbk = nblocks(tot_all, WG);
    if (S.B == 8) {
      if (dtype == SCOCG_C128)
        hipLaunchKernelGGL((k_gather_out<8, double2>), dim3(nbk), dim3(WG), 0, h->stream,
                           S.x.as<double2>(), static_cast<double2*>(d), S.K, S.R, S.nS, S.sym);
      else
        hipLaunchKernelGGL((k_gather_out<8, float2>), dim3(nbk), dim3(WG), 0, h->stream,
                           S.x.as<double2>(), static_cast<float2*>(d), S.K, S.R, S.nS, S.sym);
    } else {
      if (dtype == SCOCG_C128)
        hipLaunchKernelGGL((k_gather_out<16, double2>), dim3(nbk), dim3(WG), 0, h->stream,
                           S.x.as<double2>(), static_cast<double2*>(d), S.K, S.R, S.nS, S.sym);
      else
        hipLaunchKernelGGL((k_gather_out<16, float2>), dim3(nbk), dim3(WG), 0, h->stream,
                           S.x.as<double2>(), static_cast<float2*>(d), S.K, S.R, S.nS, S.sym);
    }
    KCHK();
    if (staged)
      HIPCHK(hipMemcpyAsync(dst, d, tot * esz,
                            dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                            h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return SCOCG_OK;
  });
}

int scocg_apply_h(scocg_handle h, const void* x_dev, void* y_dev) {
  return guarded([&]() -> int {
    require(h != nullptr && x_dev != nullptr && y_dev != nullptr, "NULL argument");
    HIPCHK(hipSetDevice(h->device));
    if (h->precision == SCOCG_FP64)
      apply_h_impl<double, 8>(*h, x_dev, y_dev);
    else
      apply_h_impl<float, 16>(*h, x_dev, y_dev);
    return SCOCG_OK;
  });
}

int scocg_apply_h_noalloc(scocg_handle h, const void* x_dev, void* y_dev) {
  return guarded([&]() -> int {
    require(h != nullptr && x_dev != nullptr && y_dev != nullptr, "NULL argument");
    HIPCHK(hipSetDevice(h->device));
    char* ws = scratch_of(h->device);
    const size_t need = h->precision == SCOCG_FP64 ? ApplyWs<double, 8>(*h).bytes
                                                   : ApplyWs<float, 16>(*h).bytes;
    require(need <= (size_t)SCOCG_SCRATCH_BYTES,
            "grid too large for the allocation-free apply: needs " + std::to_string(need) +
                " bytes of scratch, the maximum is " + std::to_string((size_t)SCOCG_SCRATCH_BYTES));
    if (h->precision == SCOCG_FP64)
      apply_h_run<double, 8>(*h, x_dev, y_dev, ws);
    else
      apply_h_run<float, 16>(*h, x_dev, y_dev, ws);
    return SCOCG_OK;
  });
}

int scocg_stream_probe(scocg_handle h, int32_t mode, int32_t nontemporal, void* buf,
                       int64_t bytes, int32_t reps, double* gbs) {
  return guarded([&]() -> int {
    require(h != nullptr && buf != nullptr && gbs != nullptr, "NULL argument");
    require(mode >= 0 && mode <= 2, "mode must be 0, 1 or 2");
    require(reps >= 1 && bytes >= 3 * 4096, "need reps >= 1 and at least 12 KiB");
    HIPCHK(hipSetDevice(h->device));
    require_device_range(buf, (size_t)bytes, h->device, "buf");
    // three equal arrays of n 16-byte vectors (a, b, c) plus one double per workgroup
    constexpr int U = 4;
    const int grid = 256 * 8;
    const int64_t n = ((bytes - grid * 8) / 3) / 16;
    require(n >= 256, "buffer too small");
    double2* a = static_cast<double2*>(buf);
    double2* b = a + n;
    double2* c = b + n;
    double* sink = reinterpret_cast<double*>(c + n);
    auto launch = [&]() {
#define SCOCG_STREAM(NR, NT)                                                                  \
  hipLaunchKernelGGL((k_stream<NR, NT, U>), dim3(grid), dim3(256), 0, h->stream, a, b, c, n, \
                     sink)
      if (mode == 0) { if (nontemporal) SCOCG_STREAM(1, true); else SCOCG_STREAM(1, false); }
      else if (mode == 1) { if (nontemporal) SCOCG_STREAM(2, true); else SCOCG_STREAM(2, false); }
      else { if (nontemporal) SCOCG_STREAM(0, true); else SCOCG_STREAM(0, false); }
#undef SCOCG_STREAM
      KCHK();
    };
    HIPCHK(hipMemsetAsync(buf, 0, (size_t)bytes, h->stream));
    launch();  // warm
    Event e0, e1;
    HIPCHK(hipEventRecord(e0, h->stream));
    for (int r = 0; r < reps; ++r) launch();
    HIPCHK(hipEventRecord(e1, h->stream));
    const double ms = elapsed_ms(e0, e1);
    const double moved = (double)n * 16 * (mode == 0 ? 2 : mode == 1 ? 3 : 1) * reps;
    *gbs = moved / (ms * 1e-3) / 1e9;
    return SCOCG_OK;
  });
}

int scocg_obm(scocg_handle h, int32_t K, int32_t M, int32_t L, const void* g_dev,
              const void* sig_l_dev, const void* sig_r_dev, void* gt_dev, double* trans,
              double* dos, double* phase_ms) {
  return guarded([&]() -> int {
    require(h != nullptr, "handle is NULL");
    require(K >= 1 && K <= 16383, "K must be in 1..16383");
    require(M >= 1 && L >= 0, "need M >= 1 and L >= 0");
    const int64_t D = 2 * (int64_t)M + L;
    require(D + 2 * (int64_t)M <= 65535 * 8, "2M + D too large for one grid row");
    HIPCHK(hipSetDevice(h->device));
    const size_t gbytes = sizeof(double2) * (size_t)K * D * D;
    const size_t sbytes = sizeof(double2) * (size_t)K * M * M;
    require_device_range(g_dev, gbytes, h->device, "g_dev");
    require_device_range(sig_l_dev, sbytes, h->device, "sig_l_dev");
    require_device_range(sig_r_dev, sbytes, h->device, "sig_r_dev");
    DevBuf own;
    double2* gt = static_cast<double2*>(gt_dev);
    if (gt_dev) {
      require_device_range(gt_dev, gbytes, h->device, "gt_dev");
      auto apart = [&](const void* x, size_t xb, const char* what) {
        const char* a = static_cast<const char*>(gt_dev);
        const char* b = static_cast<const char*>(x);
        require(a + gbytes <= b || b + xb <= a, std::string("gt_dev overlaps ") + what);
      };
      apart(g_dev, gbytes, "g_dev");
      apart(sig_l_dev, sbytes, "sig_l_dev");
      apart(sig_r_dev, sbytes, "sig_r_dev");
    } else {
      own.alloc(gbytes);
      gt = own.as<double2>();
    }
    std::vector<double2> T;
    std::vector<double> ds;
    const int nfail = obm_run(*h, K, M, L, static_cast<const double2*>(g_dev),
                              static_cast<const double2*>(sig_l_dev),
                              static_cast<const double2*>(sig_r_dev), gt, T, ds, phase_ms);
    if (trans)
      for (int k = 0; k < K; ++k) {
        trans[2 * k] = T[k].x;
        trans[2 * k + 1] = T[k].y;
      }
    if (dos)
      for (int k = 0; k < K; ++k) dos[k] = ds[k];
    if (nfail) {
      g_err = std::to_string(nfail) + " energies met a zero pivot (I - G Sigma singular)";
      return SCOCG_BREAKDOWN;
    }
    return SCOCG_OK;
  });
}

void scocg_destroy(scocg_handle h) {
  if (!h) return;
  (void)hipSetDevice(h->device);
  (void)hipStreamSynchronize(h->stream);
  hipStream_t s = h->own_stream ? h->stream : nullptr;
  delete h;
  if (s) (void)hipStreamDestroy(s);
}

const char* scocg_last_error(void) { return g_err.c_str(); }

int64_t scocg_struct_size(int32_t which) {
  switch (which) {
    case 0: return (int64_t)sizeof(scocg_grid);
    case 1: return (int64_t)sizeof(scocg_solve_opts);
    case 2: return (int64_t)sizeof(scocg_report);
    case 3: return (int64_t)sizeof(scocg_problem);
    default: return 0;
  }
}

}  // extern "C"
