// Device code of the coupled TRT-LBM / FFT-Poisson electroconvection step
// for gfx950 (wave64).  Every kernel is templated on the storage type T
// (double, or float for the FP32-deviation mode); quantities that the
// precision policy keeps in FP64 (the x-mean Poisson mode, its field, the
// reductions) are double in both modes.
//
// Data layout (row-major, x fastest):
//   populations  [9][ny][P] deviations from the hydrostatic reference rows:
//                f_i - w_i rho_ref(y) and g_i - R_i(y), R_i = w_i r(y)
//   potential    phi fluctuation [ny][P] (the m >= 1 modes) plus the x-mean
//                row in FP64
//   spectrum     [ny][MP] complex, m = 0 .. nx/2 (one row per y)
#include "ec_internal.hpp"

namespace ec {

// ---------------------------------------------------------------- complex
template <typename T>
struct C2 {
  T re, im;
};
template <typename T>
__device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) {
  return {a.re + b.re, a.im + b.im};
}
template <typename T>
__device__ __forceinline__ C2<T> csub(C2<T> a, C2<T> b) {
  return {a.re - b.re, a.im - b.im};
}
template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ C2<T> cscale(C2<T> a, T s) {
  return {a.re * s, a.im * s};
}
// multiply by s*i, s = -1 for the forward transform, +1 for the inverse
template <typename T, bool INV>
__device__ __forceinline__ C2<T> rot(C2<T> a) {
  return INV ? C2<T>{-a.im, a.re} : C2<T>{a.im, -a.re};
}

// ------------------------------------------------- small DFTs in registers
// y_q = sum_r v_r exp(s 2 pi i r q / R), s = -1 forward / +1 inverse.
template <typename T, bool INV>
__device__ __forceinline__ void dft2(C2<T>* v) {
  C2<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
template <typename T, bool INV>
__device__ __forceinline__ void dft4(C2<T>& a0, C2<T>& a1, C2<T>& a2, C2<T>& a3) {
  C2<T> t0 = cadd(a0, a2), t1 = csub(a0, a2);
  C2<T> t2 = cadd(a1, a3), t3 = rot<T, INV>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a1 = cadd(t1, t3);
  a2 = csub(t0, t2);
  a3 = csub(t1, t3);
}
template <typename T, bool INV>
__device__ __forceinline__ void dft3(C2<T>* v) {
  const T h = T(0.86602540378443864676);  // sqrt(3)/2
  C2<T> t = cadd(v[1], v[2]);
  C2<T> d = csub(v[1], v[2]);
  C2<T> y0 = cadd(v[0], t);
  C2<T> m = {v[0].re - T(0.5) * t.re, v[0].im - T(0.5) * t.im};
  C2<T> k = rot<T, INV>(cscale(d, h));
  v[0] = y0;
  v[1] = cadd(m, k);
  v[2] = csub(m, k);
}
template <typename T, bool INV>
__device__ __forceinline__ void dft5(C2<T>* v) {
  const T c1 = T(0.30901699437494742410);   // cos(2 pi / 5)
  const T c2 = T(-0.80901699437494742410);  // cos(4 pi / 5)
  const T s1 = T(0.95105651629515357212);   // sin(2 pi / 5)
  const T s2 = T(0.58778525229247312917);   // sin(4 pi / 5)
  C2<T> t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
  C2<T> t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
  C2<T> y0 = cadd(v[0], cadd(t1, t2));
  C2<T> b1 = {v[0].re + c1 * t1.re + c2 * t2.re, v[0].im + c1 * t1.im + c2 * t2.im};
  C2<T> b2 = {v[0].re + c2 * t1.re + c1 * t2.re, v[0].im + c2 * t1.im + c1 * t2.im};
  C2<T> e1 = rot<T, INV>(C2<T>{s1 * t3.re + s2 * t4.re, s1 * t3.im + s2 * t4.im});
  C2<T> e2 = rot<T, INV>(C2<T>{s2 * t3.re - s1 * t4.re, s2 * t3.im - s1 * t4.im});
  v[0] = y0;
  v[1] = cadd(b1, e1);
  v[4] = csub(b1, e1);
  v[2] = cadd(b2, e2);
  v[3] = csub(b2, e2);
}
template <typename T, bool INV>
__device__ __forceinline__ void dft8(C2<T>* v) {
  const T r = T(0.70710678118654752440);
  C2<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  C2<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<T, INV>(e0, e1, e2, e3);
  dft4<T, INV>(o0, o1, o2, o3);
  // o_q *= exp(s 2 pi i q / 8)
  const T sg = INV ? T(1) : T(-1);
  o1 = cmul(o1, C2<T>{r, sg * r});
  o2 = rot<T, INV>(o2);
  o3 = cmul(o3, C2<T>{-r, sg * r});
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1);
  v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2);
  v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3);
  v[7] = csub(e3, o3);
}

// One Stockham autosort pass of radix R (R in {2,3,4,5,8}) from src to dst:
// butterfly t reads src[t + r N/R] (r = 0..R-1) with the pre-twiddles
// exp(s 2 pi i r k / (Ns R)), k = t mod Ns, and writes its R outputs to
// dst[(t / Ns) Ns R + k + q Ns].  Ns is the product of the radices of the
// earlier passes; the last pass leaves natural order.
template <typename T, bool INV, int R>
__device__ __forceinline__ void stockham_pass(const C2<T>* __restrict__ src, C2<T>* __restrict__ dst,
                                              int N, int Ns, const C2<T>* __restrict__ twp) {
  const int stride = N / R;
  for (int t = threadIdx.x; t < stride; t += blockDim.x) {
    const int k = t % Ns;
    const C2<T>* tk = twp + k * (R - 1);
    C2<T> v[R];
    v[0] = src[t];
#pragma unroll
    for (int r = 1; r < R; ++r) {
      C2<T> w = tk[r - 1];
      if (INV) w.im = -w.im;
      v[r] = cmul(src[t + r * stride], w);
    }
    if constexpr (R == 2) dft2<T, INV>(v);
    if constexpr (R == 3) dft3<T, INV>(v);
    if constexpr (R == 4) dft4<T, INV>(v[0], v[1], v[2], v[3]);
    if constexpr (R == 5) dft5<T, INV>(v);
    if constexpr (R == 8) dft8<T, INV>(v);
    const int base = (t / Ns) * Ns * R + k;
#pragma unroll
    for (int q = 0; q < R; ++q) dst[base + q * Ns] = v[q];
  }
}

// Pass of any other radix R: a direct DFT of the R inputs per output (q, t)
// with the combined twiddle exp(s 2 pi i r (k N/(Ns R) + q N/R) / N).  Each
// output's sum is split at h = (R + 1) / 2: terms 0 .. h-1 by a thread of the
// block's first half, terms h .. R-1 by its partner in the second half, each
// in order, then added (the same order whatever the block size; the chain of
// dependent terms per thread is halved, and a transform shorter than the
// block keeps both halves busy).
template <typename T, bool INV>
__device__ __forceinline__ void generic_pass(const C2<T>* __restrict__ src, C2<T>* __restrict__ dst,
                                             int N, int Ns, int R, const C2<T>* __restrict__ tw) {
  const int stride = N / R;
  const int twstep = N / (Ns * R);
  const int h = (R + 1) / 2;
  const int half = blockDim.x / 2;
  const bool side = threadIdx.x >= half;
  const int lo = threadIdx.x - (side ? half : 0);
  for (int ob = 0; ob < N; ob += half) {
    const int o = ob + lo;
    C2<T> acc = {T(0), T(0)};
    int pos = 0;
    if (o < N) {
      const int q = o / stride;
      const int t = o - q * stride;
      const int k = t % Ns;
      const int e = (k * twstep + q * stride) % N;
      const int r0 = side ? h : 1, r1 = side ? R : h;
      int idx = (e * r0) % N;
      if (!side) acc = src[t];
#pragma unroll 4
      for (int r = r0; r < r1; ++r) {
        C2<T> w = tw[idx];
        if (INV) w.im = -w.im;
        acc = cadd(acc, cmul(src[t + r * stride], w));
        idx += e;
        if (idx >= N) idx -= N;
      }
      pos = (t / Ns) * Ns * R + k + q * Ns;
      if (side) dst[pos] = acc;
    }
    __syncthreads();
    if (o < N && !side) dst[pos] = cadd(acc, dst[pos]);
  }
}

// Complex transform of length pl.n held in LDS buffer a (b is scratch of the
// same size).  Returns the buffer that holds the result.  Unnormalised:
// forward uses exp(-2 pi i m x / N), inverse exp(+2 pi i m x / N).
template <typename T, bool INV>
__device__ __forceinline__ C2<T>* fft_lds(C2<T>* a, C2<T>* b, const FftPlan& pl, const C2<T>* __restrict__ tw) {
  const int N = pl.n;
  int Ns = 1, off = 0;
  const C2<T>* twp = tw + N;  // pass-major twiddles follow the full table
  C2<T>* src = a;
  C2<T>* dst = b;
  for (int p = 0; p < pl.nr; ++p) {
    const int R = pl.r[p];
    switch (R) {
      case 2: stockham_pass<T, INV, 2>(src, dst, N, Ns, twp + off); break;
      case 3: stockham_pass<T, INV, 3>(src, dst, N, Ns, twp + off); break;
      case 4: stockham_pass<T, INV, 4>(src, dst, N, Ns, twp + off); break;
      case 5: stockham_pass<T, INV, 5>(src, dst, N, Ns, twp + off); break;
      case 8: stockham_pass<T, INV, 8>(src, dst, N, Ns, twp + off); break;
      default: generic_pass<T, INV>(src, dst, N, Ns, R, tw); break;
    }
    if (R == 2 || R == 3 || R == 4 || R == 5 || R == 8) off += Ns * (R - 1);
    __syncthreads();
    C2<T>* tmp = src;
    src = dst;
    dst = tmp;
    Ns *= R;
  }
  return src;
}

// In-place pass of radix R (see fft_in_place): every thread holds up to NB
// butterflies of the pass in registers between the read and the write phase.
template <typename T, bool INV, int R, int NB>
__device__ __forceinline__ void stockham_pass_ip(C2<T>* __restrict__ buf, int N, int Ns,
                                                 const C2<T>* __restrict__ twp) {
  const int stride = N / R;
  C2<T> v[NB][R];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int t = threadIdx.x + q * blockDim.x;
    if (t < stride) {
      const int k = t % Ns;
      const C2<T>* tk = twp + k * (R - 1);
      v[q][0] = buf[t];
#pragma unroll
      for (int r = 1; r < R; ++r) {
        C2<T> w = tk[r - 1];
        if (INV) w.im = -w.im;
        v[q][r] = cmul(buf[t + r * stride], w);
      }
      if constexpr (R == 2) dft2<T, INV>(v[q]);
      if constexpr (R == 3) dft3<T, INV>(v[q]);
      if constexpr (R == 4) dft4<T, INV>(v[q][0], v[q][1], v[q][2], v[q][3]);
      if constexpr (R == 5) dft5<T, INV>(v[q]);
      if constexpr (R == 8) dft8<T, INV>(v[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int t = threadIdx.x + q * blockDim.x;
    if (t < stride) {
      const int k = t % Ns;
      const int base = (t / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[base + r * Ns] = v[q][r];
    }
  }
}

// The same transform as fft_lds, in place in buffer a (requires
// fft_in_place(pl, blockDim.x, F)); passes p0 .. p1-1 only (p1 < 0: to the
// end), the earlier ones done elsewhere.
template <typename T, bool INV, int F>
__device__ __forceinline__ C2<T>* fft_lds_ip(C2<T>* a, const FftPlan& pl, const C2<T>* __restrict__ tw, int p0 = 0,
                                             int p1 = -1) {
  const int N = pl.n;
  int Ns = 1;
  const C2<T>* twp = tw + N;
  for (int p = 0; p < p0; ++p) {
    twp += Ns * (pl.r[p] - 1);
    Ns *= pl.r[p];
  }
  const int pe = p1 < 0 ? pl.nr : p1;
  for (int p = p0; p < pe; ++p) {
    const int R = pl.r[p];
    switch (R) {
      case 2: stockham_pass_ip<T, INV, 2, (F + 1) / 2>(a, N, Ns, twp); break;
      case 3: stockham_pass_ip<T, INV, 3, (F + 2) / 3>(a, N, Ns, twp); break;
      case 4: stockham_pass_ip<T, INV, 4, (F + 3) / 4>(a, N, Ns, twp); break;
      case 5: stockham_pass_ip<T, INV, 5, (F + 4) / 5>(a, N, Ns, twp); break;
      default: stockham_pass_ip<T, INV, 8, (F + 7) / 8>(a, N, Ns, twp); break;
    }
    twp += Ns * (R - 1);
    __syncthreads();
    Ns *= R;
  }
  return a;
}

// Row-sum scratch of k_forward: two rows of one FP64 sum per 64-element
// group (nx <= 8192).
constexpr int kSumGroups = 128;
// In place: one buffer of n elements plus the row-sum scratch.  Ping-pong:
// two buffers, the second one doubling as the scratch (used before the
// transform starts).
template <typename T>
size_t fft_lds_bytes(const FftPlan& pl, int threads) {
  const size_t one = (size_t)pl.n * sizeof(C2<T>);
  const size_t red = 2 * kSumGroups * sizeof(double);
  if (fft_in_place(pl, threads)) return one + red;
  return one + (one > red ? one : red);
}
template size_t fft_lds_bytes<double>(const FftPlan&, int);
template size_t fft_lds_bytes<float>(const FftPlan&, int);

// Ten rows of tw values; six of them with a halo slot at each end when the
// tile is narrower than the row.
template <typename T>
size_t collide_lds_bytes(int tw, int nx) {
  return (10 * (size_t)tw + (tw < nx ? 12 : 0)) * sizeof(T);
}
template size_t collide_lds_bytes<double>(int, int);
template size_t collide_lds_bytes<float>(int, int);

// ------------------------------------------------------------- reductions
// The value of lane (lane xor O) of a wave, O in {1, 2, 4, 8, 16, 32},
// without the LDS crossbar: quad permutations (1, 2) and row shifts (4, 8)
// of DPP, and the gfx950 row / half-wave swaps (16, 32).  The same values as
// a xor shuffle.
template <int O>
__device__ __forceinline__ unsigned lane_xor(unsigned v) {
  const int lane = threadIdx.x & 63;
  if constexpr (O == 1) {
    return (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  } else if constexpr (O == 2) {
    return (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  } else if constexpr (O == 4 || O == 8) {
    const unsigned up = (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x100 + O, 0xF, 0xF, false);  // row_shl:O
    const unsigned dn = (unsigned)__builtin_amdgcn_mov_dpp((int)v, 0x110 + O, 0xF, 0xF, false);  // row_shr:O
    return (lane & O) ? dn : up;
  } else if constexpr (O == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return ((lane >> 4) & 1) ? r[0] : r[1];
  } else {
    static_assert(O == 32, "lane distance");
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return lane >= 32 ? r[0] : r[1];
  }
}
template <int O>
__device__ __forceinline__ double lane_xor(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = lane_xor<O>((unsigned)u), hi = lane_xor<O>((unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Butterfly sum over the 64 lanes (distances 32, 16, ..., 1); every lane
// gets the sum, in an order that depends only on the lane values.
__device__ __forceinline__ double wave_sum(double v) {
  v += lane_xor<32>(v);
  v += lane_xor<16>(v);
  v += lane_xor<8>(v);
  v += lane_xor<4>(v);
  v += lane_xor<2>(v);
  v += lane_xor<1>(v);
  return v;
}

// Sum of v over the block (blockDim.x a multiple of 64, <= 1024); every
// thread gets the result.  `red` holds 16 doubles of LDS.
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += red[w];
  return s;
}

// ----------------------------------------------------------- pull helpers
__device__ __forceinline__ int wrap_m(int x, int nx) { return x == 0 ? nx - 1 : x - 1; }
__device__ __forceinline__ int wrap_p(int x, int nx) { return x == nx - 1 ? 0 : x + 1; }

// Streaming load: each population is read once per step, so it should not
// displace the smaller fields (potential, spectrum, charge sums) from L2.
template <typename T>
__device__ __forceinline__ T ldnt(const T* p) {
  return __builtin_nontemporal_load(p);
}

// The pulls below choose their source addresses with selects instead of
// branches, so that all nine loads of a node are issued before the first one
// is used (branches around loads serialise them on memory latency).  Offsets
// inside a plane fit 32 bits (nx ny <= 2^31 and P < nx + 64).

// Pre-collision charge populations at (x, j), pulled from the post-collision
// deviations G with the electrode conditions (Table I read as: injector
// anti-bounce-back fixing rho_c = rho0, collector zero normal gradient).
// G holds the x movers already shifted by their c_ix: plane i at column x
// holds g*_i(x - c_ix) for i = 1, 5, 8 (c_ix = +1) and 3, 6, 7 (c_ix = -1),
// planes 0, 2, 4 hold g*_i(x) (the collide tile stores them so, from the
// values it keeps in LDS for the charge sums).  The streamed populations are
// then read at the node's own column, aligned; only the injector row's
// reflections of the same node's g*_7, g*_8 read one column aside.
template <typename T>
__device__ __forceinline__ void pull_g(const Consts& c, const T* __restrict__ G, const T* __restrict__ rows,
                                       int x, int j, T g[9]) {
  const size_t plane = (size_t)c.ny * c.P;
  const int xm = wrap_m(x, c.nx), xp = wrap_p(x, c.nx);
  const bool lo = j > 0, hi = j < c.ny - 1;
  const unsigned row = (unsigned)j * (unsigned)c.P;
  const unsigned rb = lo ? row - c.P : row, ra = hi ? row + c.P : row;
  // below the node: streamed from row j-1, or reflected at the injector
  const T* p2 = G + (lo ? 2 : 4) * plane;
  const T* p5 = G + (lo ? 5 : 7) * plane;
  const T* p6 = G + (lo ? 6 : 8) * plane;
  const unsigned o2 = rb + x, o5 = rb + (lo ? x : xm), o6 = rb + (lo ? x : xp);
  // above the node: streamed from row j+1, or the same-row neighbours at the
  // collector (zero normal gradient)
  const unsigned o4 = ra + x, o7 = ra + x, o8 = ra + x;
  const T a0 = ldnt(&G[row + x]);
  const T a1 = ldnt(&G[plane + row + x]);
  const T a3 = ldnt(&G[3 * plane + row + x]);
  const T a2 = ldnt(&p2[o2]), a5 = ldnt(&p5[o5]), a6 = ldnt(&p6[o6]);
  const T a4 = ldnt(&G[4 * plane + o4]), a7 = ldnt(&G[7 * plane + o7]), a8 = ldnt(&G[8 * plane + o8]);
  const T ua = rows[ROW_DG_UP_AXIS * c.ny + j], ud = rows[ROW_DG_UP_DIAG * c.ny + j];
  const T da = rows[ROW_DG_DN_AXIS * c.ny + j], dd = rows[ROW_DG_DN_DIAG * c.ny + j];
  g[0] = a0;
  g[1] = a1;
  g[3] = a3;
  g[2] = lo ? a2 + ua : -a2 + T(c.g_abb_axis);
  g[5] = lo ? a5 + ud : -a5 + T(c.g_abb_diag);
  g[6] = lo ? a6 + ud : -a6 + T(c.g_abb_diag);
  g[4] = hi ? a4 + da : a4;
  g[7] = hi ? a7 + dd : a7;
  g[8] = hi ? a8 + dd : a8;
}

// Pre-collision fluid populations at (x, j) with halfway bounce-back at both
// electrodes (Table I).  On the deviations from the hydrostatic fixed point
// neither the row crossings nor the walls add a constant.
template <typename T>
__device__ __forceinline__ void pull_f(const Consts& c, const T* __restrict__ F, int x, int j, T f[9]) {
  const size_t plane = (size_t)c.ny * c.P;
  const int xm = wrap_m(x, c.nx), xp = wrap_p(x, c.nx);
  const bool lo = j > 0, hi = j < c.ny - 1;
  const unsigned row = (unsigned)j * (unsigned)c.P;
  const unsigned rb = lo ? row - c.P : row, ra = hi ? row + c.P : row;
  const T* p2 = F + (lo ? 2 : 4) * plane;
  const T* p5 = F + (lo ? 5 : 7) * plane;
  const T* p6 = F + (lo ? 6 : 8) * plane;
  const T* p4 = F + (hi ? 4 : 2) * plane;
  const T* p7 = F + (hi ? 7 : 5) * plane;
  const T* p8 = F + (hi ? 8 : 6) * plane;
  f[0] = ldnt(&F[row + x]);
  f[1] = ldnt(&F[plane + row + xm]);
  f[3] = ldnt(&F[3 * plane + row + xp]);
  f[2] = ldnt(&p2[rb + x]);
  f[5] = ldnt(&p5[rb + (lo ? xm : x)]);
  f[6] = ldnt(&p6[rb + (lo ? xp : x)]);
  f[4] = ldnt(&p4[ra + x]);
  f[7] = ldnt(&p7[ra + (hi ? xp : x)]);
  f[8] = ldnt(&p8[ra + (hi ? xm : x)]);
}

template <typename T>
__device__ __forceinline__ void local_pop(const Consts& c, const T* __restrict__ A, int x, int j, T a[9]) {
  const size_t plane = (size_t)c.ny * c.P;
  const size_t idx = (size_t)j * c.P + x;
#pragma unroll
  for (int i = 0; i < 9; ++i) a[i] = A[i * plane + idx];
}

// The post-collision charge populations g*_i(x, j) of node (x, j) from G as
// the collide stores it (x movers at column x + c_ix; see pull_g).
template <typename T>
__device__ __forceinline__ void local_post_g(const Consts& c, const T* __restrict__ G, int x, int j, T a[9]) {
  const size_t plane = (size_t)c.ny * c.P;
  const size_t row = (size_t)j * c.P;
  const int xm = wrap_m(x, c.nx), xp = wrap_p(x, c.nx);
  const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
#pragma unroll
  for (int i = 0; i < 9; ++i) a[i] = G[i * plane + row + (cx[i] > 0 ? xp : (cx[i] < 0 ? xm : x))];
}

// Where the forward transform takes the charge density deviation rho_c - r
// of the step from.
template <typename T>
struct ChargeSrc {
  const T* rq;          // MODE 0: the collide tiles' sums (see collide_tile)
  const T* eu;          //         and their edge rows
  const T* ed;
  const T* G;           // MODE 1: populations summed at the node
  const double* field;  // MODE 2: a given FP64 field [ny][nx]
};

// rho_c - r at (x, j): MODE 0 completes the sums of the collide tiles with
// the contributions that cross the tile edges, MODE 1 sums the populations
// at the node (the initial state), MODE 2 reads the given field.
template <typename T, int MODE>
__device__ __forceinline__ T charge_at(const Consts& c, const ChargeSrc<T>& q, int x, int j) {
  if (MODE == 2) return T(q.field[(size_t)j * c.nx + x]);
  if (MODE == 1) {
    T g[9];
    local_pop<T>(c, q.G, x, j, g);
    return g[0] + g[1] + g[2] + g[3] + g[4] + g[5] + g[6] + g[7] + g[8];
  }
  T v = q.rq[(size_t)j * c.P + x];
  const int H = c.TH, b = j / H, j0 = b * H, j1 = min(j0 + H, c.ny);
  if (j == j0 && j > 0) v += q.eu[(size_t)(b - 1) * c.P + x];
  if (j == j1 - 1 && j1 < c.ny) v += q.ed[(size_t)(b + 1) * c.P + x];
  return v;
}

// FP64 row sums of the charge deviation in an order fixed by nx alone (so
// launch shapes never change results), shaped like the first transform pass
// (radix R0 = the plan's first radix, stride n / R0): the partial P(t) =
// sum_r a[t + r n / R0] in order of r for t < n / R0; the partials of each
// aligned group of 64 (t = 64 g + l) summed across the lanes of one wave by
// the butterfly of wave_sum; the groups g = l, l + 64 in order by lane l of
// one wave, then again by wave_sum.  Every path below gives each wave whole
// aligned groups of t (blockDim is a multiple of 64).
// group_sums: lane 0 of the wave stores the group sums of a row pair.
__device__ __forceinline__ void group_sums(double v0, double v1, int g, double* red) {
  v0 = wave_sum(v0);
  v1 = wave_sum(v1);
  if ((threadIdx.x & 63) == 0) {
    red[g] = v0;
    red[kSumGroups + g] = v1;
  }
}

// After a barrier that follows group_sums: wave 0 combines the G groups,
// thread 0 stores the row sums.
__device__ __forceinline__ void combine_groups(const double* red, int G, double* __restrict__ dcsum, int j0,
                                               bool has1) {
  if (threadIdx.x < 64) {
    double s0 = 0.0, s1 = 0.0;
    for (int g = threadIdx.x; g < G; g += 64) {
      s0 += red[g];
      s1 += red[kSumGroups + g];
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    if (threadIdx.x == 0) {
      dcsum[j0] = s0;
      if (has1) dcsum[j0 + 1] = s1;
    }
  }
}

// ------------------------------------------- forward transform (with gather)
// One block per pair of rows (j0 = 2 b, j1 = 2 b + 1) packed as the real and
// imaginary parts of one complex transform.  Writes the source spectrum
// s_m = -DFT(rho_c - r)_m / eps for m = 1 .. nx/2 (Eq. 4, 19) and the FP64
// row sums of the charge deviation (the m = 0 mode).
//
// When each thread holds exactly NB radix-8 butterflies of the first pass
// (nx = 8 NB blockDim, in place), the loaded values go through that pass in
// registers (thread t loads x = t + blockDim i, i = q + 8 NB r for butterfly q
// and input r: the stride-nx/8 inputs of the first Stockham pass), which
// saves a round trip through LDS and a barrier; the arithmetic is that of the
// LDS pass.
template <typename T, int MODE, int NB>
__device__ __forceinline__ void forward_first_pass(const Consts& c, const ChargeSrc<T>& q, const C2<T>* __restrict__ tw,
                                                   C2<T>* __restrict__ a, double* red, int j0, int j1c, bool has1) {
  constexpr int R = 8;
  const int B = blockDim.x, t = threadIdx.x, wbase = t & ~63;
  const int N = c.nx;
  C2<T> v[NB][R];
#pragma unroll
  for (int qq = 0; qq < NB; ++qq)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int x = t + B * (qq + NB * r);
      v[qq][r] = C2<T>{charge_at<T, MODE>(c, q, x, j0), charge_at<T, MODE>(c, q, x, j1c)};
    }
#pragma unroll
  for (int qq = 0; qq < NB; ++qq) {
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (!has1) v[qq][r].im = T(0);
      s0 += (double)v[qq][r].re;
      s1 += (double)v[qq][r].im;
    }
    group_sums(s0, s1, (wbase + B * qq) >> 6, red);
  }
  // first pass: Ns = 1, so k = 0 and the butterfly of t' = t + B q writes 8 t' + r
  const C2<T>* twp = tw + N;
#pragma unroll
  for (int qq = 0; qq < NB; ++qq) {
#pragma unroll
    for (int r = 1; r < R; ++r) v[qq][r] = cmul(v[qq][r], twp[r - 1]);
    dft8<T, false>(v[qq]);
    const int tp = t + B * qq;
#pragma unroll
    for (int r = 0; r < R; ++r) a[R * tp + r] = v[qq][r];
  }
}

template <typename T, int MODE, int F>
__device__ __forceinline__ void forward_body(const Consts& c, const ChargeSrc<T>& q, const FftPlan& pl,
                                             const C2<T>* __restrict__ tw, C2<T>* __restrict__ spec,
                                             double* __restrict__ dcsum, int bx) {
  extern __shared__ __align__(16) unsigned char smem[];
  C2<T>* a = reinterpret_cast<C2<T>*>(smem);
  C2<T>* b = a + pl.n;  // second transform buffer, or only the scratch when in place
  double* red = reinterpret_cast<double*>(b);  // row-sum groups (idle until the transform)
  const bool ip = fft_in_place(pl, blockDim.x, F);
  const int j0 = 2 * bx, j1 = j0 + 1;
  const bool has1 = j1 < c.ny;
  const int j1c = has1 ? j1 : j0;  // a missing second row re-reads the first; dropped below
  const int R0 = pl.nr > 0 ? pl.r[0] : 1;
  const int S = pl.n / R0;  // partials of the row sums
  const int G = (S + 63) >> 6;
  const int B = blockDim.x;
  int p0 = 0;
  if (ip && pl.r[0] == 8 && c.nx == 8 * B) {
    forward_first_pass<T, MODE, 1>(c, q, tw, a, red, j0, j1c, has1);
    p0 = 1;
  } else if (F >= 16 && ip && pl.r[0] == 8 && c.nx == 16 * B) {
    forward_first_pass<T, MODE, (F >= 16 ? 2 : 1)>(c, q, tw, a, red, j0, j1c, has1);
    p0 = 1;
  } else {
    // U columns per thread per round: every load of a round is issued before
    // the first sum (the column index is clamped, the stores are guarded);
    // the rounds are uniform over a wave (its lanes hold one aligned group)
    constexpr int U = 4;
    const int lane = threadIdx.x & 63;
    for (int xb = threadIdx.x - lane; xb < c.nx; xb += U * B) {
      T v0[U], v1[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int x = min(xb + lane + u * B, c.nx - 1);
        v0[u] = charge_at<T, MODE>(c, q, x, j0);
        v1[u] = charge_at<T, MODE>(c, q, x, j1c);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int x = xb + lane + u * B;
        if (x < c.nx) a[x] = C2<T>{v0[u], has1 ? v1[u] : T(0)};
      }
    }
    __syncthreads();
    for (int tb = threadIdx.x - lane; tb < S; tb += B) {
      const int t = tb + lane;
      double s0 = 0.0, s1 = 0.0;
      if (t < S)
        for (int r = 0; r < R0; ++r) {
          const C2<T> z = a[t + r * S];
          s0 += (double)z.re;
          s1 += (double)z.im;
        }
      group_sums(s0, s1, tb >> 6, red);
    }
  }
  __syncthreads();
  combine_groups(red, G, dcsum, j0, has1);
  if (!ip) __syncthreads();  // the ping-pong transform overwrites the group sums
  C2<T>* z = ip ? fft_lds_ip<T, false, F>(a, pl, tw, p0) : fft_lds<T, false>(a, b, pl, tw);
  const T sc = T(-0.5 / c.eps);
  const int N = pl.n;
  for (int m = threadIdx.x; m < c.M; m += blockDim.x) {
    C2<T> X = {T(0), T(0)}, Y = {T(0), T(0)};
    if (m > 0) {
      const C2<T> zm = z[m], zn = z[N - m];
      // X = (Z_m + conj Z_{N-m}) / 2,  Y = (Z_m - conj Z_{N-m}) / (2 i)
      X = C2<T>{(zm.re + zn.re) * sc, (zm.im - zn.im) * sc};
      Y = C2<T>{(zm.im + zn.im) * sc, (zn.re - zm.re) * sc};
    }
    spec[(size_t)j0 * c.MP + m] = X;
    if (has1) spec[(size_t)j1 * c.MP + m] = Y;
  }
}

// Waves per SIMD that the register allocation of the transform kernels
// aims at.  FP32 transforms with 8 elements per thread are held to 64
// registers (a few spill slots in the inverse), so that four 512-thread
// blocks share a CU instead of two or three: measured faster at 4096 points
// (forward 54 -> 49 us, inverse 54 -> 44 us).  The wider instantiations
// keep the compiler's choice.
template <typename T, int F>
struct TransformWaves {
  static constexpr int value = (sizeof(T) == 4 && F == 8) ? 8 : 1;
};

template <typename T, int MODE, int F>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(TransformWaves<T, F>::value))) k_forward(Consts c, ChargeSrc<T> q, FftPlan pl, const C2<T>* __restrict__ tw,
                                                 C2<T>* __restrict__ spec, double* __restrict__ dcsum) {
  forward_body<T, MODE, F>(c, q, pl, tw, spec, dcsum, blockIdx.x);
}

// --------------------------------------------------- x-mean mode (m = 0)
// The x-mean potential by integrating Gauss's law twice (flux form of the
// m = 0 row of Eq. 18 / 24 with the electrode ghost rows):
//   sbar(j) = -(r(j) + dcsum(j) / nx) / eps
//   D(j) = D(-1) + S(j),  S = running sum of sbar,
//   D(-1) = (phi_upper - phi_lower)/ny - (S(ny-1) + 2 sum_{k<ny-1} S(k)) / (2 ny)
//   phi_mean(j) = phi_lower + D(-1)/2 + sum_{k<j} D(k),  E_y mean = -(D(j) + D(j-1))/2
// One block; FP64 throughout.
// The column is swept in chunks of kMeanRows * 64 rows, one wave per chunk
// (each lane holds kMeanRows consecutive rows in registers); the block takes
// its waves' chunks in rounds.  Running sums: inclusive shuffle scans of the
// lane partials inside a chunk, and the chunk totals added strictly in chunk
// order, so every sum has an order fixed by ny alone (launch shapes never
// change results).  A first sweep finds S(ny-1) and the sum of S, hence
// D(-1); the second one writes the rows.  Both sweeps form S(j) by the same
// operations, so they agree exactly.  Two rows per lane keep the inverse
// transform kernel, which runs this as its block 0, within its 64 registers
// without spills.
constexpr int kMeanRows = 2;

// Inclusive scan over the lanes of a wave (in lane order, Hillis-Steele).
__device__ __forceinline__ double wave_incl_scan(double x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const double y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

__device__ __forceinline__ void mean_mode_body(const Consts& c, double* __restrict__ rowsd,
                                               double* __restrict__ dmean) {
  __shared__ double tot[16], aux[16];
  const int ny = c.ny;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  constexpr int CR = 64 * kMeanRows;
  const int nchunks = (ny + CR - 1) / CR;
  const double* r = rowsd + ROWD_R * ny;
  const double* dcs = rowsd + ROWD_DCSUM * ny;
  const double inx = (double)c.nx;
  // sbar(j) = -(r(j) + dcsum(j) / nx) / eps; S(j) = sum_{k <= j} sbar(k)
  double carry = 0.0;  // S before the round's first chunk
  double Ttot = 0.0;   // sum_{k < ny-1} S(k), chunk by chunk
  for (int c0 = 0; c0 < nchunks; c0 += nw) {
    const int ch = c0 + wave;
    const int lo = ch * CR + lane * kMeanRows;
    double sb[kMeanRows];
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < kMeanRows; ++q) {
      const int j = min(lo + q, ny - 1);
      const double v = -(r[j] + dcs[j] / inx) / c.eps;
      sb[q] = lo + q < ny ? v : 0.0;
      part += sb[q];
    }
    const double x = wave_incl_scan(part);
    const double xu = __shfl_up(x, 1, 64);  // every lane takes part in the shuffle
    const double ex = lane ? xu : 0.0;
    if (lane == 63) tot[wave] = ch < nchunks ? x : 0.0;
    __syncthreads();
    double cc = carry;  // S before this chunk
    for (int w = 0; w < wave; ++w) cc += tot[w];
    double S = cc + ex, ts = 0.0;
#pragma unroll
    for (int q = 0; q < kMeanRows; ++q) {
      S += sb[q];
      if (lo + q < ny - 1) ts += S;
    }
    ts = wave_sum(ts);
    if (lane == 0) aux[wave] = ch < nchunks ? ts : 0.0;
    __syncthreads();
    for (int w = 0; w < nw && c0 + w < nchunks; ++w) {
      carry += tot[w];
      Ttot += aux[w];
    }
    __syncthreads();
  }
  const double Slast = carry;
  const double dlow = (0.0 - 1.0) / (double)ny - (Slast + 2.0 * Ttot) / (2.0 * ny);
  const double phi0 = 1.0 + 0.5 * dlow;
  double* eym = rowsd + ROWD_EYM * ny;
  double* phim = rowsd + ROWD_PHIM * ny;
  double* dfy = rowsd + ROWD_DFY * ny;
  if (threadIdx.x == 0) dmean[0] = dlow;
  // D(j) = D(-1) + S(j); the potential is the exclusive running sum of D
  carry = 0.0;
  double pcarry = 0.0;  // sum of D before the round's first chunk
  for (int c0 = 0; c0 < nchunks; c0 += nw) {
    const int ch = c0 + wave;
    const int lo = ch * CR + lane * kMeanRows;
    double sb[kMeanRows], rr[kMeanRows];
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < kMeanRows; ++q) {
      const int j = min(lo + q, ny - 1);
      rr[q] = r[j];
      const double v = -(rr[q] + dcs[j] / inx) / c.eps;
      sb[q] = lo + q < ny ? v : 0.0;
      part += sb[q];
    }
    const double x = wave_incl_scan(part);
    const double xu = __shfl_up(x, 1, 64);  // every lane takes part in the shuffle
    const double ex = lane ? xu : 0.0;
    if (lane == 63) tot[wave] = ch < nchunks ? x : 0.0;
    __syncthreads();
    double cc = carry;
    for (int w = 0; w < wave; ++w) cc += tot[w];
    const double off = cc + ex;
    double S = off, D[kMeanRows], pd = 0.0;
#pragma unroll
    for (int q = 0; q < kMeanRows; ++q) {
      S += sb[q];
      D[q] = dlow + S;
      if (lo + q < ny) pd += D[q];
    }
    const double px = wave_incl_scan(pd);
    const double pxu = __shfl_up(px, 1, 64);
    const double pex = lane ? pxu : 0.0;
    if (lane == 63) aux[wave] = ch < nchunks ? px : 0.0;
    __syncthreads();
    double pc = pcarry;
    for (int w = 0; w < wave; ++w) pc += aux[w];
    double run = pc + pex;
    double Dprev = dlow + off;  // D(lo - 1); D(-1) = dlow
#pragma unroll
    for (int q = 0; q < kMeanRows; ++q) {
      const int j = lo + q;
      if (j < ny) {
        dmean[1 + j] = D[q];
        phim[j] = phi0 + run;
        const double e = -(D[q] + Dprev) / 2.0;
        eym[j] = e;
        dfy[j] = rr[q] * e - c.s_ref / 3.0;
        run += D[q];
        Dprev = D[q];
      }
    }
    for (int w = 0; w < nw && c0 + w < nchunks; ++w) {
      carry += tot[w];
      pcarry += aux[w];
    }
    __syncthreads();
  }
}

// ------------------------------------------------- per-wavenumber solves
// m = 1 .. nx/2: phi(j+1) - (2 + kappa_m^2) phi(j) + phi(j-1) = s(j) with
// homogeneous ghost closures (Eq. 20, 24-25 as a tridiagonal per m), solved
// by partition: the column splits into chunks of kChunk rows; in chunk k the
// solution is x = y + v L_k + w R_k, where y solves the chunk's own system
// with zero values outside it, v and w are the chunk's responses to unit
// values in the row just below (L_k) and just above (R_k), and L_k, R_k come
// from a 2x2 block-tridiagonal system over the chunk interfaces.

__device__ __forceinline__ int chunk_type(int k, int nc) {
  return nc == 1 ? CH_SINGLE : (k == 0 ? CH_FIRST : (k == nc - 1 ? CH_LAST : CH_INTERIOR));
}

// Table q (0 elimination factors, 1 v, 2 w) of a chunk type, row i, wavenumber m.
template <typename T>
__device__ __forceinline__ T ttab(const T* __restrict__ tt, int MP, int type, int q, int i, int m) {
  return tt[((size_t)(type * 3 + q) * kChunk + i) * MP + m];
}

// One thread per (m, chunk): elimination and back substitution of the
// chunk's own system in registers; y overwrites the spectrum, its first and
// last rows go to `ends`.
template <typename T>
__device__ __forceinline__ void tri_local_body(const Consts& c, const T* __restrict__ tt, C2<T>* __restrict__ spec,
                                               C2<T>* __restrict__ ends, int bx, int by) {
  const int m = 1 + bx * blockDim.x + threadIdx.x;
  const int k = by;
  if (m >= c.M) return;
  const int s0 = k * kChunk;
  const int len = min(kChunk, c.ny - s0);
  const int type = chunk_type(k, c.NC);
  const size_t MP = c.MP;
  // every row of the chunk is loaded before the elimination starts (row
  // index clamped: a short last chunk re-reads its last row, unused)
  C2<T> d[kChunk];
  T f[kChunk];
#pragma unroll
  for (int i = 0; i < kChunk; ++i) {
    const int ii = min(i, len - 1);
    d[i] = spec[(size_t)(s0 + ii) * MP + m];
    f[i] = ttab(tt, c.MP, type, 0, ii, m);
  }
  C2<T> prev = {T(0), T(0)};
#pragma unroll
  for (int i = 0; i < kChunk; ++i) {
    if (i < len) {
      prev = C2<T>{(d[i].re - prev.re) * f[i], (d[i].im - prev.im) * f[i]};
      d[i] = prev;
    }
  }
  C2<T> x = {T(0), T(0)}, first = {T(0), T(0)}, last = {T(0), T(0)};
#pragma unroll
  for (int i = kChunk - 1; i >= 0; --i) {
    if (i < len) {
      if (i == len - 1) {
        x = d[i];
        last = x;
      } else {
        x = C2<T>{d[i].re - f[i] * x.re, d[i].im - f[i] * x.im};
      }
      spec[(size_t)(s0 + i) * MP + m] = x;
    }
  }
  first = x;
  ends[(2 * (size_t)k) * MP + m] = first;
  ends[(2 * (size_t)k + 1) * MP + m] = last;
}

template <typename T>
__global__ void __launch_bounds__(256) k_tri_local(Consts c, const T* __restrict__ tt, C2<T>* __restrict__ spec,
                                                   C2<T>* __restrict__ ends) {
  const int b = blockIdx.x;
  const int nbx = (c.M - 1 + blockDim.x - 1) / blockDim.x;
  tri_local_body<T>(c, tt, spec, ends, b % nbx, b / nbx);
}

// One thread per m: the interface system.  Interface k (between chunks k
// and k+1) carries a_k = x(last row of chunk k) and b_k = x(first row of
// chunk k+1):
//   a_k - v_e(k) a_{k-1} - w_e(k) b_k       = y_e(k)
//   b_k - v_s(k+1) a_k   - w_s(k+1) b_{k+1} = y_s(k+1)
// (v_s, v_e, w_s, w_e: first / last entries of the chunk responses), solved
// by block elimination with 2x2 pivots [[1, beta], [gamma, 1]].
template <typename T>
__device__ __forceinline__ void tri_reduced_body(const Consts& c, const T* __restrict__ tt,
                                                 const C2<T>* __restrict__ ends, T* __restrict__ gh,
                                                 C2<T>* __restrict__ iface, int bx) {
  const int m = 1 + bx * blockDim.x + threadIdx.x;
  if (m >= c.M) return;
  const int nc = c.NC;
  if (nc < 2) return;
  const size_t MP = c.MP;
  T g01_prev = T(0);
  C2<T> h0_prev = {T(0), T(0)};
  // responses of an interior chunk (the same for every interior chunk)
  const T ve_in = nc > 2 ? ttab(tt, c.MP, CH_INTERIOR, 1, kChunk - 1, m) : T(0);
  const T we_in = nc > 2 ? ttab(tt, c.MP, CH_INTERIOR, 2, kChunk - 1, m) : T(0);
  const T vs_in = nc > 2 ? ttab(tt, c.MP, CH_INTERIOR, 1, 0, m) : T(0);
  const T ws_in = nc > 2 ? ttab(tt, c.MP, CH_INTERIOR, 2, 0, m) : T(0);
  // the first chunk has no lower response; the last one no upper response
  const T we_first = ttab(tt, c.MP, CH_FIRST, 2, kChunk - 1, m);
  const T vs_last = ttab(tt, c.MP, CH_LAST, 1, 0, m);
  // interfaces in rounds of KB: the loads of a round are issued first (the
  // elimination itself is a serial chain over k)
  constexpr int KB = 8;
  for (int k0 = 0; k0 < nc - 1; k0 += KB) {
    C2<T> yev[KB], ysv[KB];
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      const int k = min(k0 + u, nc - 2);
      yev[u] = ends[(2 * (size_t)k + 1) * MP + m];
      ysv[u] = ends[(2 * (size_t)(k + 1)) * MP + m];
    }
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      const int k = k0 + u;
      if (k < nc - 1) {
        const T ve = k == 0 ? T(0) : ve_in;
        const T we = k == 0 ? we_first : we_in;
        const T vs = k + 1 == nc - 1 ? vs_last : vs_in;
        const T ws = k + 1 == nc - 1 ? T(0) : ws_in;
        const C2<T> ye = yev[u];
        const C2<T> ys = ysv[u];
        const T beta = -we + ve * g01_prev;
        const T gamma = -vs;
        const T inv = T(1) / (T(1) - beta * gamma);
        const C2<T> D0 = {ye.re + ve * h0_prev.re, ye.im + ve * h0_prev.im};
        const C2<T> D1 = ys;
        const C2<T> H0 = {(D0.re - beta * D1.re) * inv, (D0.im - beta * D1.im) * inv};
        const C2<T> H1 = {(D1.re - gamma * D0.re) * inv, (D1.im - gamma * D0.im) * inv};
        const T g01 = beta * ws * inv;
        const T g11 = -ws * inv;
        T* q = gh + (6 * (size_t)k) * MP + m;
        q[0] = g01;
        q[MP] = g11;
        q[2 * MP] = H0.re;
        q[3 * MP] = H0.im;
        q[4 * MP] = H1.re;
        q[5 * MP] = H1.im;
        g01_prev = g01;
        h0_prev = H0;
      }
    }
  }
  C2<T> bnext = {T(0), T(0)};
#pragma unroll 8
  for (int k = nc - 2; k >= 0; --k) {
    const T* q = gh + (6 * (size_t)k) * MP + m;
    const T g01 = q[0], g11 = q[MP];
    const C2<T> a = {q[2 * MP] - g01 * bnext.re, q[3 * MP] - g01 * bnext.im};
    const C2<T> b = {q[4 * MP] - g11 * bnext.re, q[5 * MP] - g11 * bnext.im};
    iface[(2 * (size_t)k) * MP + m] = a;
    iface[(2 * (size_t)k + 1) * MP + m] = b;
    bnext = b;
  }
}

template <typename T>
__global__ void __launch_bounds__(64) k_tri_reduced(Consts c, const T* __restrict__ tt, const C2<T>* __restrict__ ends,
                                                    T* __restrict__ gh, C2<T>* __restrict__ iface) {
  tri_reduced_body<T>(c, tt, ends, gh, iface, blockIdx.x);
}

// The interface system by recursive doubling, one wave per wavenumber m.
// Its matrix does not depend on the data, so the block elimination above
// reduces, with factors precomputed per (m, k) (table rf), to two first-order
// linear recurrences over the interfaces:
//   h_k = A_k h_{k-1} + B_k,         B_k = inv_k ye_k - ib_k ys_k   (h = H0)
//   b_k = C_k b_{k+1} + H1_k,        H1_k = inv_k ys_k + P_k ye_k + Q_k h_{k-1}
//   a_k = h_k - g_k b_{k+1}
// (h_{-1} = 0, b_{NC-1} = 0).  Lane l holds interfaces l E .. l E + E - 1
// (E = kScanPerLane); each recurrence composes the affine maps of a lane,
// scans the composed maps across the 64 lanes (Hillis-Steele with shuffles)
// and re-runs the lane's own elements from the value that enters it.
template <typename T>
__device__ __forceinline__ C2<T> shfl_up_c(C2<T> v, int d) {
  return C2<T>{__shfl_up(v.re, d, 64), __shfl_up(v.im, d, 64)};
}
template <typename T>
__device__ __forceinline__ C2<T> shfl_down_c(C2<T> v, int d) {
  return C2<T>{__shfl_down(v.re, d, 64), __shfl_down(v.im, d, 64)};
}

template <typename T>
__device__ __forceinline__ void tri_scan_body(const Consts& c, const T* __restrict__ rf,
                                              const C2<T>* __restrict__ ends, C2<T>* __restrict__ iface, int m) {
  constexpr int E = kScanPerLane;
  const int lane = threadIdx.x & 63;
  const int K = c.NC - 1;
  const size_t MP = c.MP;
  const T* f = rf + (size_t)m * RF_COUNT * c.KP;
  const int k0 = lane * E;
  // all loads first (interface index clamped; unused beyond K)
  C2<T> ye[E], ys[E], H0[E], H1[E];
  T inv[E], ib[E], A[E], P[E], Q[E], Cf[E], g[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = min(k0 + e, K - 1);
    ye[e] = ends[(2 * (size_t)k + 1) * MP + m];
    ys[e] = ends[(2 * (size_t)(k + 1)) * MP + m];
    inv[e] = f[RF_INV * c.KP + k];
    ib[e] = f[RF_IB * c.KP + k];
    A[e] = f[RF_A * c.KP + k];
    P[e] = f[RF_P * c.KP + k];
    Q[e] = f[RF_Q * c.KP + k];
    Cf[e] = f[RF_C * c.KP + k];
    g[e] = f[RF_G * c.KP + k];
  }
  // forward: compose this lane's maps h -> A h + B
  T Al = T(1);
  C2<T> Bl = {T(0), T(0)};
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = k0 + e;
    if (k < K) {
      const C2<T> B = {inv[e] * ye[e].re - ib[e] * ys[e].re, inv[e] * ye[e].im - ib[e] * ys[e].im};
      Bl = C2<T>{A[e] * Bl.re + B.re, A[e] * Bl.im + B.im};
      Al = A[e] * Al;
    }
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T Ao = __shfl_up(Al, d, 64);
    const C2<T> Bo = shfl_up_c(Bl, d);
    if (lane >= d) {
      Bl = C2<T>{Al * Bo.re + Bl.re, Al * Bo.im + Bl.im};
      Al = Al * Ao;
    }
  }
  C2<T> hp = shfl_up_c(Bl, 1);  // h entering this lane (h_{-1} = 0)
  if (lane == 0) hp = C2<T>{T(0), T(0)};
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = k0 + e;
    if (k < K) {
      H1[e] = C2<T>{inv[e] * ys[e].re + P[e] * ye[e].re + Q[e] * hp.re,
                    inv[e] * ys[e].im + P[e] * ye[e].im + Q[e] * hp.im};
      const C2<T> B = {inv[e] * ye[e].re - ib[e] * ys[e].re, inv[e] * ye[e].im - ib[e] * ys[e].im};
      hp = C2<T>{A[e] * hp.re + B.re, A[e] * hp.im + B.im};
      H0[e] = hp;
    }
  }
  // backward: compose b_next -> C b_next + H1 over this lane's elements
  T Cl = T(1);
  C2<T> Dl = {T(0), T(0)};
#pragma unroll
  for (int e = E - 1; e >= 0; --e) {
    const int k = k0 + e;
    if (k < K) {
      Dl = C2<T>{Cf[e] * Dl.re + H1[e].re, Cf[e] * Dl.im + H1[e].im};
      Cl = Cf[e] * Cl;
    }
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T Co = __shfl_down(Cl, d, 64);
    const C2<T> Do = shfl_down_c(Dl, d);
    if (lane + d < 64) {
      Dl = C2<T>{Cl * Do.re + Dl.re, Cl * Do.im + Dl.im};
      Cl = Cl * Co;
    }
  }
  C2<T> bn = shfl_down_c(Dl, 1);  // b leaving this lane upwards (b_{NC-1} = 0)
  if (lane == 63) bn = C2<T>{T(0), T(0)};
#pragma unroll
  for (int e = E - 1; e >= 0; --e) {
    const int k = k0 + e;
    if (k < K) {
      const C2<T> a = {H0[e].re - g[e] * bn.re, H0[e].im - g[e] * bn.im};
      const C2<T> b = {H1[e].re + Cf[e] * bn.re, H1[e].im + Cf[e] * bn.im};
      iface[(2 * (size_t)k) * MP + m] = a;
      iface[(2 * (size_t)k + 1) * MP + m] = b;
      bn = b;
    }
  }
}

// Four wavenumbers per 256-thread block.  Each wave reads one wavenumber's
// column of the chunk ends (one element per interface row), so the blocks
// take their wavenumbers in the XCD-aware order (see xcd_order): the blocks
// that share the cache lines of neighbouring wavenumbers sit on one XCD and
// meet in its L2.
__device__ __forceinline__ int xcd_order(int b, int G);
template <typename T>
__global__ void __launch_bounds__(256) k_tri_scan(Consts c, const T* __restrict__ rf, const C2<T>* __restrict__ ends,
                                                  C2<T>* __restrict__ iface) {
  const int m = 1 + xcd_order(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (m >= c.M) return;
  tri_scan_body<T>(c, rf, ends, iface, m);
}

// Solved spectra of a row pair in LDS: the chunk-local y (in spec) plus the
// responses v, w to the interface values L (below the chunk) and R (above
// it).  Both rows of a pair lie in one chunk (kChunk is even), so the
// presence of L and R is uniform over the block and is resolved by the
// template outside the loop; the loads of a round carry no branches.
template <typename T, bool HL, bool HR>
__device__ __forceinline__ void inverse_gather(const Consts& c, const C2<T>* __restrict__ spec,
                                               const T* __restrict__ tt, const C2<T>* __restrict__ iface,
                                               int j0, bool has1, int N, C2<T>* __restrict__ a) {
  const size_t MP = c.MP;
  const int k = j0 / kChunk, i0 = j0 - k * kChunk;
  const int type = chunk_type(k, c.NC);
  const C2<T>* y0 = spec + (size_t)j0 * MP;
  const C2<T>* y1 = spec + (size_t)(has1 ? j0 + 1 : j0) * MP;
  const T* v0 = tt + ((size_t)(type * 3 + 1) * kChunk + i0) * MP;
  const T* w0 = tt + ((size_t)(type * 3 + 2) * kChunk + i0) * MP;
  const int i1 = has1 ? i0 + 1 : i0;
  const T* v1 = tt + ((size_t)(type * 3 + 1) * kChunk + i1) * MP;
  const T* w1 = tt + ((size_t)(type * 3 + 2) * kChunk + i1) * MP;
  const C2<T>* Lp = iface + (2 * (size_t)(HL ? k - 1 : 0)) * MP;
  const C2<T>* Rp = iface + (2 * (size_t)k + 1) * MP;
  // the lower half m < M is loaded once; the upper half N - m holds the
  // conjugates (the two rows are real)
  constexpr int U = 4;
  const int M = c.M;
  for (int m0 = threadIdx.x; m0 < M; m0 += U * blockDim.x) {
    C2<T> X[U], Y[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int m = min(m0 + u * (int)blockDim.x, M - 1);
      X[u] = y0[m];
      Y[u] = y1[m];
      if (HL) {
        const C2<T> L = Lp[m];
        const T a0 = v0[m], a1 = v1[m];
        X[u].re += a0 * L.re;
        X[u].im += a0 * L.im;
        Y[u].re += a1 * L.re;
        Y[u].im += a1 * L.im;
      }
      if (HR) {
        const C2<T> R = Rp[m];
        const T b0 = w0[m], b1 = w1[m];
        X[u].re += b0 * R.re;
        X[u].im += b0 * R.im;
        Y[u].re += b1 * R.re;
        Y[u].im += b1 * R.im;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int m = m0 + u * (int)blockDim.x;
      if (m < M) {
        const C2<T> x = X[u], y = has1 ? Y[u] : C2<T>{T(0), T(0)};
        a[m] = m == 0 ? C2<T>{T(0), T(0)} : C2<T>{x.re - y.im, x.im + y.re};
        if (m >= 1 && N - m >= M) a[N - m] = C2<T>{x.re + y.im, y.re - x.im};
      }
    }
  }
}

// Last pass (radix R, Ns = n / R) of an in-place inverse transform, its
// outputs scaled by inv and stored as the real / imaginary parts to two
// potential rows instead of to LDS (the same arithmetic as stockham_pass_ip).
template <typename T, int R, int NB>
__device__ __forceinline__ void inverse_last_pass(const C2<T>* __restrict__ buf, const FftPlan& pl,
                                                  const C2<T>* __restrict__ tw, int last, T inv, T* __restrict__ phi0,
                                                  T* __restrict__ phi1, bool has1) {
  const int N = pl.n;
  const int stride = N / R;
  const C2<T>* twp = tw + N;
  for (int p = 0, Ns = 1; p < last; ++p) {
    twp += Ns * (pl.r[p] - 1);
    Ns *= pl.r[p];
  }
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int t = threadIdx.x + q * blockDim.x;
    if (t < stride) {
      // k = t % Ns = t, base = t
      const C2<T>* tk = twp + t * (R - 1);
      C2<T> v[R];
      v[0] = buf[t];
#pragma unroll
      for (int r = 1; r < R; ++r) {
        C2<T> w = tk[r - 1];
        w.im = -w.im;
        v[r] = cmul(buf[t + r * stride], w);
      }
      if constexpr (R == 2) dft2<T, true>(v);
      if constexpr (R == 3) dft3<T, true>(v);
      if constexpr (R == 4) dft4<T, true>(v[0], v[1], v[2], v[3]);
      if constexpr (R == 5) dft5<T, true>(v);
      if constexpr (R == 8) dft8<T, true>(v);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int x = t + r * stride;
        phi0[x] = v[r].re * inv;
        if (has1) phi1[x] = v[r].im * inv;
      }
    }
  }
}

// --------------------------------------------------- inverse transform
// Pair of rows per block: Z_m = X_m + i Y_m with the Hermitian halves of the
// two solved spectra (m = 0 left out: it lives in the x-mean row), inverse
// transform, 1/nx, real / imaginary parts to the two rows of phi.
template <typename T, int F>
__device__ __forceinline__ void inverse_body(const Consts& c, const C2<T>* __restrict__ spec,
                                             const T* __restrict__ tt, const C2<T>* __restrict__ iface,
                                             const FftPlan& pl, const C2<T>* __restrict__ tw, T* __restrict__ phi,
                                             int bx) {
  extern __shared__ __align__(16) unsigned char smem[];
  C2<T>* a = reinterpret_cast<C2<T>*>(smem);
  C2<T>* b = a + pl.n;
  const int j0 = 2 * bx, j1 = j0 + 1;
  const bool has1 = j1 < c.ny;
  const int N = pl.n;
  const int k = j0 / kChunk;
  const bool hl = c.NC > 1 && k > 0, hr = c.NC > 1 && k < c.NC - 1;
  if (hl && hr)
    inverse_gather<T, true, true>(c, spec, tt, iface, j0, has1, N, a);
  else if (hl)
    inverse_gather<T, true, false>(c, spec, tt, iface, j0, has1, N, a);
  else if (hr)
    inverse_gather<T, false, true>(c, spec, tt, iface, j0, has1, N, a);
  else
    inverse_gather<T, false, false>(c, spec, tt, iface, j0, has1, N, a);
  __syncthreads();
  const T inv = T(1.0 / (double)N);
  T* phi0 = phi + (size_t)j0 * c.P;
  T* phi1 = phi + (size_t)(has1 ? j1 : j0) * c.P;
  if (fft_in_place(pl, blockDim.x, F) && pl.nr > 0) {
    // all passes but the last in LDS; the last one stores straight to the
    // potential rows (its butterfly t < n / R writes x = t + (n / R) r)
    const int last = pl.nr - 1;
    fft_lds_ip<T, true, F>(a, pl, tw, 0, last);
    switch (pl.r[last]) {
      case 2: inverse_last_pass<T, 2, (F + 1) / 2>(a, pl, tw, last, inv, phi0, phi1, has1); break;
      case 3: inverse_last_pass<T, 3, (F + 2) / 3>(a, pl, tw, last, inv, phi0, phi1, has1); break;
      case 4: inverse_last_pass<T, 4, (F + 3) / 4>(a, pl, tw, last, inv, phi0, phi1, has1); break;
      case 5: inverse_last_pass<T, 5, (F + 4) / 5>(a, pl, tw, last, inv, phi0, phi1, has1); break;
      default: inverse_last_pass<T, 8, (F + 7) / 8>(a, pl, tw, last, inv, phi0, phi1, has1); break;
    }
    return;
  }
  C2<T>* z = fft_in_place(pl, blockDim.x, F) ? a : fft_lds<T, true>(a, b, pl, tw);
  for (int x = threadIdx.x; x < c.nx; x += blockDim.x) {
    phi0[x] = z[x].re * inv;
    if (has1) phi1[x] = z[x].im * inv;
  }
}

// Block 0 solves the x-mean mode (needed only by the collision, and
// independent of the m >= 1 modes, so it runs beside the transforms);
// blocks 1.. are the row pairs, taken in the XCD-aware order (see
// xcd_order), so that the sixteen row pairs of a 32-row chunk, which read the
// same interface values and chunk responses, sit on one XCD and share them
// in its L2.
__device__ __forceinline__ int xcd_order(int b, int G);
template <typename T, int F>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(TransformWaves<T, F>::value))) k_inverse(Consts c, const C2<T>* __restrict__ spec, const T* __restrict__ tt,
                                                 const C2<T>* __restrict__ iface, FftPlan pl,
                                                 const C2<T>* __restrict__ tw, T* __restrict__ phi,
                                                 double* __restrict__ rowsd, double* __restrict__ dmean) {
  if (blockIdx.x == 0) {
    mean_mode_body(c, rowsd, dmean);
    return;
  }
  inverse_body<T, F>(c, spec, tt, iface, pl, tw, phi, xcd_order(blockIdx.x - 1, gridDim.x - 1));
}

// Workgroups are dealt to the eight XCDs in turn; block b takes index
// start(b mod 8) + b / 8, start(x) = x q + min(x, r) for G = 8 q + r blocks (a
// bijection onto 0 .. G-1), so that the blocks of one XCD take consecutive
// indices and share their cache lines in that XCD's L2.
__device__ __forceinline__ int xcd_order(int b, int G) {
  const int q = G >> 3, r = G & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}

// ------------------------------------------- fused collide (and stream)
// One thread per node.  PULL: gathers the pre-collision populations from the
// post-collision arrays with the wall rules (the streaming of Eq. 8-9);
// otherwise reads them at the node (first collision of the initial state).
// Then the moments (Eq. 5-7), E = -grad phi (central differences, the mean
// row in FP64), the equilibria (Eq. 10-11), the source (Eq. 12) and the TRT
// collisions (Eq. 8-9, 13-15); writes the post-collision deviations.
// mom == nullptr: no moments are emitted.  STORE false: nothing is written
// (a halo column of an x-tile, whose node belongs to the neighbouring tile).
// gout receives the post-collision charge populations as stored (rounded
// to T), for the charge density of the next step; of them the node stores
// g*_0, g*_2, g*_4 itself, and the tile stores the x movers, shifted (see
// pull_g and collide_tile).
template <typename T, typename C, bool PULL, bool STORE = true>
__device__ __forceinline__ void collide_node(const Consts& c, const T* __restrict__ Fin, const T* __restrict__ Gin,
                                             T* __restrict__ Fout, T* __restrict__ Gout,
                                             const T* __restrict__ phi, const T* __restrict__ rows,
                                             const double* __restrict__ rowsd, double* __restrict__ mom, int x, int j,
                                             T gout[9]) {
  // every load of the node first (populations, then the potential around
  // it), so that they are in flight together; the scheduling barrier keeps
  // the compiler from interleaving the first uses with them
  const int xm = wrap_m(x, c.nx), xp = wrap_p(x, c.nx);
  const size_t row = (size_t)j * c.P;
  const bool lo = j > 0, hi = j < c.ny - 1;
  T ft[9], gt[9];
  if (PULL) {
    pull_f<T>(c, Fin, x, j, ft);
    pull_g<T>(c, Gin, rows, x, j, gt);
  } else {
    local_pop<T>(c, Fin, x, j, ft);
    local_pop<T>(c, Gin, x, j, gt);
  }
  const T pcT = phi[row + x], pxpT = phi[row + xp], pxmT = phi[row + xm];
  const T pynT = phi[(hi ? row + c.P : row) + x], pysT = phi[(lo ? row - c.P : row) + x];
  __builtin_amdgcn_sched_barrier(0);
  C f[9], g[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    f[i] = (C)ft[i];
    g[i] = (C)gt[i];
  }
  // moments
  const C drho = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
  const C rho = (C)rows[ROW_RHO_REF * c.ny + j] + drho;
  const C jx = f[1] - f[3] + f[5] - f[6] - f[7] + f[8];
  const C jy = f[2] - f[4] + f[5] + f[6] - f[7] - f[8];
  const C drc = g[0] + g[1] + g[2] + g[3] + g[4] + g[5] + g[6] + g[7] + g[8];
  const C rc = (C)rows[ROW_R * c.ny + j] + drc;
  // electric field: central differences; the ghost rows of the fluctuation
  // potential are its odd reflections (-phi) at both walls
  const C pc = (C)pcT, pxp = (C)pxpT, pxm = (C)pxmT;
  const C pyp = hi ? (C)pynT : -pc;
  const C pym = lo ? (C)pysT : -pc;
  const C ex = C(-0.5) * (pxp - pxm);
  const C eyf = C(-0.5) * (pyp - pym);  // transverse-mode part of E_y
  const C ey = C(rowsd[ROWD_EYM * c.ny + j]) + eyf;
  const C fx = rc * ex + C(c.bx);
  // y force less the reference force s/3, without forming the large terms:
  // rho_c E_y - s/3 = (r E_y,mean - s/3) + r E_y,fluct + (rho_c - r) E_y
  const C dfy = C(rowsd[ROWD_DFY * c.ny + j]) + (C)rows[ROW_R * c.ny + j] * eyf + drc * ey;
  const C fy = C(c.s_ref / 3.0) + dfy;
  // Eq. 7 on the deviations: sum_i c_i f_ref,i = -(s/6) y-hat cancels s/3 / 2
  const C irho = C(1) / rho;
  const C ux = (jx + C(0.5) * fx) * irho;
  const C uy = (jy + C(0.5) * dfy) * irho;
  const C vx = ux + C(c.K) * ex;
  const C vy = uy + C(c.K) * ey;
  if (mom != nullptr) {
    const size_t n = (size_t)c.ny * c.nx, k = (size_t)j * c.nx + x;
    mom[k] = (double)drho;
    mom[n + k] = (double)ux;
    mom[2 * n + k] = (double)uy;
    mom[3 * n + k] = (double)drc;
  }
  // TRT on the symmetric / antisymmetric parts of each pair (i, opp):
  //   f^eq_i - w_i rho_ref = w_i drho + w_i rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u)
  //     -> symmetric w drho + w rho (4.5 (c.u)^2 - 1.5 u.u), antisymmetric w rho 3 c.u
  //   F_i = w_i [3 (c_i - u) + 9 (c_i.u) c_i] . F with its part 3 w_i c_iy s/3
  //     carried by the reference (3 c.(F - s/3 y-hat) in place of 3 c.F)
  //     -> symmetric w (9 (c.u)(c.F) - 3 u.F), antisymmetric 3 w c.(F - s/3 y-hat)
  //   charge: g^eq_i - R_i = w_i drc + w_i rc (3 c.v + 4.5 (c.v)^2 - 1.5 v.v)
  //   post-collision: f_i - [w+ (f+ - e+) - (1 - w+/2) S+] -/+ [w- (f- - e-) - (1 - w-/2) S-]
  const C w0 = C(4.0 / 9.0), wa = C(1.0 / 9.0), wd = C(1.0 / 36.0);
  const C wp = C(c.wp), wm = C(c.wm), wgp = C(c.wgp), wgm = C(c.wgm);
  const C sp = C(1) - C(0.5) * wp, sm = C(1) - C(0.5) * wm;
  const C uu15 = C(1.5) * (ux * ux + uy * uy);
  const C vv15 = C(1.5) * (vx * vx + vy * vy);
  const C uF = ux * fx + uy * fy;
  const size_t plane = (size_t)c.ny * c.P;
  const size_t idx = row + x;
  // streaming stores: the populations are read again only next step
  auto put = [&](int i, C fv, C gv) {
    gout[i] = (T)gv;
    if constexpr (STORE) {
      __builtin_nontemporal_store((T)fv, &Fout[i * plane + idx]);
      if (i == 0 || i == 2 || i == 4) __builtin_nontemporal_store(gout[i], &Gout[i * plane + idx]);
    }
  };
  // With FP32 collision arithmetic the rest populations close each
  // lattice's post-collision sum onto its pre-collision moment (the TRT step
  // conserves mass and charge, and the source sums to zero), so that the
  // rounding of the FP32 equilibria does not accumulate in rho and rho_c;
  // with FP64 arithmetic the rest direction relaxes like the others.
  constexpr bool kClose = sizeof(C) == 4;
  C fs = C(0), gs = C(0);
  if constexpr (!kClose) {  // rest direction
    const C feq0 = w0 * drho - (w0 * rho) * uu15;
    const C F0 = -(C(3) * w0) * uF;
    const C geq0 = w0 * drc - (w0 * rc) * vv15;
    put(0, f[0] - wp * (f[0] - feq0) + sp * F0, g[0] - wgp * (g[0] - geq0));
  }
  const int pi[4] = {1, 2, 5, 6}, po[4] = {3, 4, 7, 8};
  const C cxs[4] = {C(1), C(0), C(1), C(-1)}, cys[4] = {C(0), C(1), C(1), C(1)};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = pi[q], o = po[q];
    const C w = q < 2 ? wa : wd;
    const C cx = cxs[q], cy = cys[q];
    const C cu = cx * ux + cy * uy;
    const C cv = cx * vx + cy * vy;
    const C cF = cx * fx + cy * fy;
    const C cdF = cx * fx + cy * dfy;
    const C wr = w * rho, wc = w * rc;
    const C ep = w * drho + wr * (C(4.5) * cu * cu - uu15);
    const C em = wr * (C(3) * cu);
    const C Sp = w * (C(9) * cu * cF - C(3) * uF);
    const C Sm = (C(3) * w) * cdF;
    const C fp = C(0.5) * (f[i] + f[o]), fm = C(0.5) * (f[i] - f[o]);
    const C A = wp * (fp - ep) - sp * Sp;
    const C B = wm * (fm - em) - sm * Sm;
    const C hp = w * drc + wc * (C(4.5) * cv * cv - vv15);
    const C hm = wc * (C(3) * cv);
    const C gp = C(0.5) * (g[i] + g[o]), gm = C(0.5) * (g[i] - g[o]);
    const C Ag = wgp * (gp - hp);
    const C Bg = wgm * (gm - hm);
    const C fi = (f[i] - A) - B, fo = (f[o] - A) + B, gi = (g[i] - Ag) - Bg, go = (g[o] - Ag) + Bg;
    put(i, fi, gi);
    put(o, fo, go);
    if constexpr (kClose) {
      fs += fi + fo;
      gs += gi + go;
    }
  }
  if constexpr (kClose) put(0, drho - fs, drc - gs);
}

// One block per tile of rows [j0, j1) and columns [x0, x0 + tw): it collides
// the rows in order and forms, from the post-collision charge populations it
// has just written, the charge density the next step's pull will see,
// rho_c^{n+1}(x, j) = sum_i g*_i(x - c_i, j - c_iy) with the electrode rules
// of Table I and the re-reference constants of the deviations (k_q(j), one
// per row).  Row r contributes
//   S(x) = g*_0(x) + g*_1(x-1) + g*_3(x+1)      to row r,
//   U(x) = g*_2(x) + g*_5(x-1) + g*_6(x+1)      to row r+1,
//   D(x) = g*_4(x) + g*_8(x-1) + g*_7(x+1)      to row r-1;
// the injector row takes -(g*_4 + g*_7 + g*_8)(x) (anti-bounce-back, same
// node) in place of U from below, the collector row takes its own D in place
// of D from above.  The x neighbours come through LDS; the y direction is
// marched.  A tile of whole rows (tw = nx) wraps x inside the block; a
// narrower tile also collides its two halo columns x0 - 1 and x0 + tw (the
// neighbouring tiles' nodes, recomputed from the same inputs, so bit for bit
// the values those tiles write) and keeps only their x movers.  Every node's
// sum has the same expression in any tile width, so the width is free to
// tune.  Written: rq (the density of rows j0 .. j1-1, without U from row
// j0-1 and without D from row j1), eu[b] = U of row j1-1 and ed[b] = D of row
// j0 (the forward transform adds them across the tile edges).  All sums in
// T, in a fixed order.  The x movers of G are stored from LDS already shifted
// (column x receives g*_1, g*_5, g*_8 of x - 1 and g*_3, g*_6, g*_7 of x + 1),
// the values the sums read there anyway: the next pull then reads every
// plane at the node's column, and loads that straddle cache lines (which the
// streaming loads do not keep for the neighbouring wave) are avoided for
// those six planes.
//
// LDS: the six x movers of the current row (in a narrower tile with a halo
// slot at each end), own g*_4, the incomplete P of the current and of the
// previous row, U.
// DENS: no collision; g* is read from Gin as stored (the density of a state
// whose post-collision populations were changed in place); nothing else is
// written.
template <typename T, typename C, bool PULL, bool EMIT, bool DENS = false>
__device__ __forceinline__ void collide_tile(const Consts& c, const T* __restrict__ Fin, const T* __restrict__ Gin,
                                             T* __restrict__ Fout, T* __restrict__ Gout, const T* __restrict__ phi,
                                             const T* __restrict__ rows, const double* __restrict__ rowsd,
                                             double* __restrict__ mom, T* __restrict__ rq, T* __restrict__ eu,
                                             T* __restrict__ ed, int blk) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nx = c.nx, ny = c.ny;
  const int ntx = collide_xtiles(c);
  const int b = blk / ntx;               // row band
  const int x0 = (blk - b * ntx) * c.TW;  // first column
  const int tw = min(c.TW, nx - x0);
  const bool whole = tw == nx;
  // mover slots: whole rows wrap inside the block; a narrower tile keeps
  // column x0 - 1 + k in slot k
  const int W = whole ? tw : tw + 2;
  const int so = whole ? 0 : 1;  // slot of column x0 + xl is xl + so
  T* L = reinterpret_cast<T*>(smem);
  T* m1 = L;            // g*_1, g*_5, g*_8 move to x+1
  T* m5 = L + W;
  T* m8 = L + 2 * W;
  T* m3 = L + 3 * W;    // g*_3, g*_6, g*_7 move to x-1
  T* m6 = L + 4 * W;
  T* m7 = L + 5 * W;
  T* o4 = L + 6 * W;    // own g*_4
  T* Pa = o4 + tw;      // P of rows r and r-1 (swapped every row)
  T* Pb = Pa + tw;
  T* Ua = Pb + tw;      // U of the previous row, then of the current one
  const int H = c.TH;
  const int j0 = b * H, j1 = min(j0 + H, ny);
  const T* kq = rows + ROW_KQ * ny;
  const int slots = whole ? tw : tw + 2;
  for (int r = j0; r < j1; ++r) {
    T* Pcur = ((r - j0) & 1) ? Pb : Pa;   // P(r) being built
    T* Pprev = ((r - j0) & 1) ? Pa : Pb;  // P(r-1), complete
    for (int q = threadIdx.x; q < slots; q += blockDim.x) {
      // q < tw: column x0 + q of the tile; then the halo columns x0 - 1, x0 + tw
      const int xl = q < tw ? q : (q == tw ? -1 : tw);
      int x = x0 + xl;
      x = x < 0 ? x + nx : (x >= nx ? x - nx : x);
      T gt[9];
      if constexpr (DENS) {
        local_post_g<T>(c, Gin, x, r, gt);
      } else {
        if (q < tw)
          collide_node<T, C, PULL>(c, Fin, Gin, Fout, Gout, phi, rows, rowsd, EMIT ? mom : nullptr, x, r, gt);
        else
          collide_node<T, C, PULL, false>(c, Fin, Gin, Fout, Gout, phi, rows, rowsd, nullptr, x, r, gt);
      }
      m1[xl + so] = gt[1];
      m5[xl + so] = gt[5];
      m8[xl + so] = gt[8];
      m3[xl + so] = gt[3];
      m6[xl + so] = gt[6];
      m7[xl + so] = gt[7];
      if (q < tw) {
        o4[xl] = gt[4];
        const T below = r == 0 ? -(gt[4] + gt[7] + gt[8]) : (r > j0 ? Ua[xl] : T(0));
        Pcur[xl] = (below + gt[0]) + kq[r];
        Ua[xl] = gt[2];
      }
    }
    __syncthreads();
    for (int xl = threadIdx.x; xl < tw; xl += blockDim.x) {
      const int x = x0 + xl;
      // slots of the columns xl - 1 and xl + 1
      const int sm = whole ? (xl == 0 ? tw - 1 : xl - 1) : xl;
      const int sp = whole ? (xl == tw - 1 ? 0 : xl + 1) : xl + 2;
      const T D = (o4[xl] + m8[sm]) + m7[sp];
      if (r > j0)
        rq[(size_t)(r - 1) * c.P + x] = Pprev[xl] + D;
      else if (r > 0)
        ed[(size_t)b * c.P + x] = D;
      if constexpr (!DENS) {
        const size_t pl = (size_t)ny * c.P, k = (size_t)r * c.P + x;
        __builtin_nontemporal_store(m1[sm], &Gout[pl + k]);
        __builtin_nontemporal_store(m5[sm], &Gout[5 * pl + k]);
        __builtin_nontemporal_store(m8[sm], &Gout[8 * pl + k]);
        __builtin_nontemporal_store(m3[sp], &Gout[3 * pl + k]);
        __builtin_nontemporal_store(m6[sp], &Gout[6 * pl + k]);
        __builtin_nontemporal_store(m7[sp], &Gout[7 * pl + k]);
      }
      const T P = (Pcur[xl] + m1[sm]) + m3[sp];
      const T U = (Ua[xl] + m5[sm]) + m6[sp];
      Pcur[xl] = P;
      Ua[xl] = U;
      if (r == j1 - 1) {
        rq[(size_t)r * c.P + x] = r == ny - 1 ? P + D : P;
        if (r < ny - 1) eu[(size_t)b * c.P + x] = U;
      }
    }
    __syncthreads();
  }
}

template <typename T, typename C, bool PULL, bool EMIT>
__global__ void __launch_bounds__(1024) k_collide(Consts c, const T* __restrict__ Fin, const T* __restrict__ Gin,
                                                  T* __restrict__ Fout, T* __restrict__ Gout,
                                                  const T* __restrict__ phi, const T* __restrict__ rows,
                                                  const double* __restrict__ rowsd, double* __restrict__ mom,
                                                  T* __restrict__ rq, T* __restrict__ eu, T* __restrict__ ed) {
  collide_tile<T, C, PULL, EMIT>(c, Fin, Gin, Fout, Gout, phi, rows, rowsd, mom, rq, eu, ed, blockIdx.x);
}

// Spectral y solve (Eq. 21-25), one block per x wavenumber m >= 1: the
// column s_m(j) of the spectrum is extended oddly about the half-cell walls
// to length N = 2 ny (entry N - 1 - j holds -s_m(j)), transformed, divided
// by the symbol -(kappa_m^2 + 4 sin^2(pi k / N)) of the 3-point y difference
// with the electrode ghosts and the spectral x derivative, transformed back
// (1 / N), and the first ny entries overwrite the column: the same solution
// as the tridiagonal systems, reached the paper's way.  The column is read
// and written at the spectrum's row pitch (one element per row).
template <typename T>
__global__ void __launch_bounds__(256) k_yspec(Consts c, FftPlan py, const C2<T>* __restrict__ twy,
                                               C2<T>* __restrict__ spec) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int N = py.n, ny = c.ny;
  C2<T>* a = reinterpret_cast<C2<T>*>(smem);
  C2<T>* b = a + N;
  const int m = 1 + xcd_order(blockIdx.x, gridDim.x);  // neighbouring columns share cache lines
  const size_t MP = c.MP;
  for (int j = threadIdx.x; j < ny; j += blockDim.x) {
    const C2<T> v = spec[(size_t)j * MP + m];
    a[j] = v;
    a[N - 1 - j] = C2<T>{-v.re, -v.im};
  }
  __syncthreads();
  C2<T>* r = fft_lds<T, false>(a, b, py, twy);
  const int mf = min(m, c.nx - m);
  const double kap = 2.0 * (double)mf / (double)c.nx;  // kappa_m / pi
  for (int k = threadIdx.x; k < N; k += blockDim.x) {
    const double sn = sinpi((double)k / (double)N);
    const double sym = -(M_PI * M_PI * kap * kap + 4.0 * sn * sn);
    const T f = (T)(1.0 / (sym * (double)N));
    r[k] = cscale(r[k], f);
  }
  __syncthreads();
  C2<T>* o = fft_lds<T, true>(r, r == a ? b : a, py, twy);
  for (int j = threadIdx.x; j < ny; j += blockDim.x) spec[(size_t)j * MP + m] = o[j];
}

// The same with the in-place transform, for columns whose length has only
// register radices and at most kFftPerThread elements per thread of 512: one
// column buffer in LDS, so that two blocks share a CU where the ping-pong
// form fits one.
template <typename T>
__global__ void __launch_bounds__(512) k_yspec_ip(Consts c, FftPlan py, const C2<T>* __restrict__ twy,
                                                  C2<T>* __restrict__ spec) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int N = py.n, ny = c.ny;
  C2<T>* a = reinterpret_cast<C2<T>*>(smem);
  const int m = 1 + xcd_order(blockIdx.x, gridDim.x);  // neighbouring columns share cache lines
  const size_t MP = c.MP;
  for (int j = threadIdx.x; j < ny; j += blockDim.x) {
    const C2<T> v = spec[(size_t)j * MP + m];
    a[j] = v;
    a[N - 1 - j] = C2<T>{-v.re, -v.im};
  }
  __syncthreads();
  fft_lds_ip<T, false, kFftPerThread>(a, py, twy);
  const int mf = min(m, c.nx - m);
  const double kap = 2.0 * (double)mf / (double)c.nx;  // kappa_m / pi
  for (int k = threadIdx.x; k < N; k += blockDim.x) {
    const double sn = sinpi((double)k / (double)N);
    const double sym = -(M_PI * M_PI * kap * kap + 4.0 * sn * sn);
    a[k] = cscale(a[k], (T)(1.0 / (sym * (double)N)));
  }
  __syncthreads();
  fft_lds_ip<T, true, kFftPerThread>(a, py, twy);
  for (int j = threadIdx.x; j < ny; j += blockDim.x) spec[(size_t)j * MP + m] = a[j];
}

// The tiles' charge density sums from the stored post-collision g*.
template <typename T>
__global__ void __launch_bounds__(1024) k_density(Consts c, const T* __restrict__ G, const T* __restrict__ rows,
                                                  T* __restrict__ rq, T* __restrict__ eu, T* __restrict__ ed) {
  collide_tile<T, T, false, false, true>(c, nullptr, G, nullptr, nullptr, nullptr, rows, nullptr, nullptr, rq, eu,
                                         ed, blockIdx.x);
}

// Continuation at another T (one thread per node), in FP64:
//  * the full post-collision charge populations R_i + g_i are scaled by
//    `scale` (the ratio of the new charge unit eps / H^2 to the old one) and
//    re-referenced to the new rows, g_i <- scale g_i + w_i (scale r_old -
//    r_new); the charge moment (rho_c - r of the last step) likewise;
//  * the fluid populations keep their departure from the hydrostatic state
//    w_i (rho_ref + c_iy s / 2), s its force slope.  The stored deviations
//    already are that departure when the reference rows use s itself; where
//    they use s rounded for the storage type (s_T = s + delta), they move by
//    -w_i (delta_new - delta_old) (y_c + c_iy / 2), y_c = j + 1/2 - H/2, and
//    the density moment by -(delta_new - delta_old) y_c.  ddelta = delta_new -
//    delta_old (zero in FP64 storage, where nothing is rewritten).
template <typename T>
__global__ void __launch_bounds__(256) k_continue(Consts c, T* __restrict__ F, T* __restrict__ G,
                                                  double* __restrict__ mom, const double* __restrict__ rowsd,
                                                  double scale, double ddelta) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (x >= c.nx) return;
  const double d = scale * rowsd[ROWD_R * c.ny + j] - rowsd[ROWD_RNEXT * c.ny + j];
  const double wv[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                        1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
  const double cyv[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  const size_t plane = (size_t)c.ny * c.P, idx = (size_t)j * c.P + x;
#pragma unroll
  for (int i = 0; i < 9; ++i) G[i * plane + idx] = (T)(scale * (double)G[i * plane + idx] + wv[i] * d);
  const size_t n = (size_t)c.ny * c.nx, k = (size_t)j * c.nx + x;
  mom[3 * n + k] = scale * mom[3 * n + k] + d;
  if (ddelta != 0.0) {
    const double yc = ((double)j + 0.5) - 0.5 * c.H;
#pragma unroll
    for (int i = 0; i < 9; ++i)
      F[i * plane + idx] = (T)((double)F[i * plane + idx] - wv[i] * ddelta * (yc + 0.5 * cyv[i]));
    mom[k] -= ddelta * yc;
  }
}

// ------------------------------------------------------------ init kernels
__device__ __forceinline__ double splitmix_uniform_pm1(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  const double u = (double)(z >> 11) * 0x1.0p-53;
  return 2.0 * u - 1.0;
}

// Initial charge deviation rho_c^0 - r into mom plane 3 (FP64).
template <typename T>
__global__ void __launch_bounds__(256) k_init_charge(Consts c, const double* __restrict__ rowsd, double* __restrict__ mom) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (x >= c.nx) return;
  const size_t n = (size_t)c.ny * c.nx, k = (size_t)j * c.nx + x;
  const double rcl = rowsd[ROWD_RC_CLOSED * c.ny + j];
  double rc0 = rcl;
  if (c.init_mode == 0) {
    const double xi = splitmix_uniform_pm1(c.seed, k);
    rc0 = rcl * (1.0 + c.noise_amp * xi);
  }
  mom[3 * n + k] = rc0 - rowsd[ROWD_R * c.ny + j];
}

// Pre-collision equilibria of the initial state at the nodes of buffer dst:
// f^0 = f^eq(rho_ref, u^0), g^0 = g^eq(rho_c^0, u^0 + K E^0), E^0 from the
// potential just solved for rho_c^0.  u^0 = 0, or the Eq. 29 perturbation.
template <typename T>
__global__ void __launch_bounds__(256) k_init_populations(Consts c, T* __restrict__ F, T* __restrict__ G,
                                                          const T* __restrict__ phi, const double* __restrict__ rowsd,
                                                          const double* __restrict__ mom) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (x >= c.nx) return;
  const size_t n = (size_t)c.ny * c.nx, k = (size_t)j * c.nx + x;
  const double drc = mom[3 * n + k];
  const double rc = rowsd[ROWD_R * c.ny + j] + drc;
  // initial density 1 + s_init (y - H/2); its difference from the reference row
  const double yc = ((double)j + 0.5) - 0.5 * c.H;
  const double rho = 1.0 + c.s_init * yc;
  const double drho0 = (c.s_init - c.s_ref) * yc;
  double ux = 0.0, uy = 0.0;
  if (c.init_mode == 1) {
    const double twopi = 6.283185307179586;
    const double Lx = (double)c.nx / (double)c.ny, Ly = 1.0;
    const double xx = (double)x / (double)c.ny, yy = ((double)j + 0.5) / (double)c.ny;
    ux = 1e-3 * c.u0 * Lx * sin(twopi * yy / Ly) * sin(twopi * xx / Lx);
    uy = 1e-3 * c.u0 * Ly * (cos(twopi * yy / Ly) - 1.0) * cos(twopi * xx / Lx);
  }
  const int xm = wrap_m(x, c.nx), xp = wrap_p(x, c.nx);
  const size_t row = (size_t)j * c.P;
  const double pc = (double)phi[row + x];
  const double pyp = j < c.ny - 1 ? (double)phi[row + c.P + x] : -pc;
  const double pym = j > 0 ? (double)phi[row - c.P + x] : -pc;
  const double ex = -((double)phi[row + xp] - (double)phi[row + xm]) / 2.0;
  const double ey = rowsd[ROWD_EYM * c.ny + j] - (pyp - pym) / 2.0;
  const double vx = ux + c.K * ex, vy = uy + c.K * ey;
  const double cxv[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  const double cyv[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  const double wv[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                        1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
  const double uu = ux * ux + uy * uy, vv = vx * vx + vy * vy;
  const size_t plane = (size_t)c.ny * c.P;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double cu = cxv[i] * ux + cyv[i] * uy;
    const double cv = cxv[i] * vx + cyv[i] * vy;
    // f^0 = w_i rho_init (1 + ...) less f_ref = w_i (rho_ref - (s/2) c_iy)
    const double fe = wv[i] * drho0 + wv[i] * rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu) +
                      0.5 * c.s_ref * wv[i] * cyv[i];
    const double ge = wv[i] * drc + wv[i] * rc * (3.0 * cv + 4.5 * cv * cv - 1.5 * vv);
    F[i * plane + row + x] = (T)fe;
    G[i * plane + row + x] = (T)ge;
  }
}

// Nondimensional FP64 output fields of the current state.  rho_m1 = rho - 1
// as (rho_ref - 1) + (rho - rho_ref): rho_ref - 1 is exact (rho_ref lies
// within a factor two of 1), so the departure keeps its relative precision.
template <typename T>
__global__ void __launch_bounds__(256) k_fields(Consts c, const double* __restrict__ mom, const T* __restrict__ phi,
                                                const double* __restrict__ rowsd, double* rho, double* ux,
                                                double* uy, double* rho_c, double* phio, double* rho_m1) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (x >= c.nx) return;
  const size_t n = (size_t)c.ny * c.nx, k = (size_t)j * c.nx + x;
  if (rho) rho[k] = rowsd[ROWD_RHO_REF * c.ny + j] + mom[k];
  if (rho_m1) rho_m1[k] = (rowsd[ROWD_RHO_REF * c.ny + j] - 1.0) + mom[k];
  if (ux) ux[k] = mom[n + k] / c.u0;
  if (uy) uy[k] = mom[2 * n + k] / c.u0;
  if (rho_c) rho_c[k] = (rowsd[ROWD_R * c.ny + j] + mom[3 * n + k]) * c.H * c.H / c.eps;
  if (phio) phio[k] = rowsd[ROWD_PHIM * c.ny + j] + (double)phi[(size_t)j * c.P + x];
}

// Charge deviation field from a nondimensional charge density (Poisson entry).
__global__ void __launch_bounds__(256) k_charge_in(Consts c, const double* __restrict__ rc_nd,
                                                   const double* __restrict__ rowsd, double* __restrict__ mom) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (x >= c.nx) return;
  const size_t n = (size_t)c.ny * c.nx, k = (size_t)j * c.nx + x;
  mom[3 * n + k] = rc_nd[k] * c.eps / (c.H * c.H) - rowsd[ROWD_R * c.ny + j];
}

// Maximum of v over the block (every thread gets it); `red` holds 16
// doubles of LDS.
__device__ double block_max(double v, double* red) {
  v = fmax(v, lane_xor<32>(v));
  v = fmax(v, lane_xor<16>(v));
  v = fmax(v, lane_xor<8>(v));
  v = fmax(v, lane_xor<4>(v));
  v = fmax(v, lane_xor<2>(v));
  v = fmax(v, lane_xor<1>(v));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double m = red[0];
  for (int w = 1; w < nw; ++w) m = fmax(m, red[w]);
  return m;
}

// Global FP64 diagnostics of the emitted moments, in two passes with a
// fixed reduction order: block b of k_stats_part reduces its band of rows
// into part[b][0..6] (sums of rho - 1, rho_c, u_y^2 and of the unhealthy
// nodes; maxima of |u|, -rho_c and |E_x|); k_stats_final reduces the bands
// in order.
template <typename T>
__global__ void __launch_bounds__(256) k_stats_part(Consts c, const double* __restrict__ mom,
                                                    const T* __restrict__ phi, const double* __restrict__ rowsd,
                                                    double* __restrict__ part) {
  __shared__ double red[16];
  const int nb = gridDim.x, b = blockIdx.x;
  const int j0 = (int)((long long)c.ny * b / nb), j1 = (int)((long long)c.ny * (b + 1) / nb);
  const size_t n = (size_t)c.ny * c.nx;
  double s_drho = 0, s_rc = 0, s_uy2 = 0, bad = 0, mx_u = 0, mx_nrc = -1e300, mx_ex = 0;
  for (int j = j0; j < j1; ++j) {
    const double r = rowsd[ROWD_R * c.ny + j], rr = rowsd[ROWD_RHO_REF * c.ny + j];
    for (int x = threadIdx.x; x < c.nx; x += blockDim.x) {
      const size_t k = (size_t)j * c.nx + x;
      const double drho = mom[k], ux = mom[n + k], uy = mom[2 * n + k];
      const double rc = r + mom[3 * n + k];
      const double rho = rr + drho;
      s_drho += (rho - 1.0);
      s_rc += rc;
      s_uy2 += uy * uy;
      mx_u = fmax(mx_u, sqrt(ux * ux + uy * uy));
      mx_nrc = fmax(mx_nrc, -rc);
      if (!(rho > 0.0) || !isfinite(rho) || !isfinite(ux) || !isfinite(uy) || !isfinite(rc)) bad += 1.0;
      const int xm = wrap_m(x, c.nx), xp = wrap_p(x, c.nx);
      const double ex = -((double)phi[(size_t)j * c.P + xp] - (double)phi[(size_t)j * c.P + xm]) / 2.0;
      mx_ex = fmax(mx_ex, fabs(ex));
    }
  }
  double v[7];
  v[0] = block_sum(s_drho, red);
  v[1] = block_sum(s_rc, red);
  v[2] = block_sum(s_uy2, red);
  v[3] = block_sum(bad, red);
  v[4] = block_max(mx_u, red);
  v[5] = block_max(mx_nrc, red);
  v[6] = block_max(mx_ex, red);
  if (threadIdx.x == 0)
    for (int q = 0; q < 7; ++q) part[8 * b + q] = v[q];
}

// The charge that the next streaming of the post-collision populations G
// moves across the electrodes (Table I): in through the injector (the
// anti-bounce-back replaces each outgoing g*_i by 2 w_i rho0 - g*_i) and net
// in through the collector (the incoming populations copy the last row, the
// outgoing ones leave).  On deviations the reference rows cancel except in
// the injector constants g_abb = 2 w_i (rho0 - r(0)).  Whole-row sums, so
// the x shift of the stored movers (see pull_g) leaves them unchanged.
template <typename T>
__global__ void __launch_bounds__(256) k_stats_final(Consts c, const double* __restrict__ part, int nb,
                                                     const T* __restrict__ G, double* __restrict__ out) {
  __shared__ double red[16];
  const size_t plane = (size_t)c.ny * c.P, top = (size_t)(c.ny - 1) * c.P;
  double q_in = 0, q_out = 0;
  for (int x = threadIdx.x; x < c.nx; x += blockDim.x) {
    q_in += (c.g_abb_axis - 2.0 * (double)G[4 * plane + x]) + (c.g_abb_diag - 2.0 * (double)G[7 * plane + x]) +
            (c.g_abb_diag - 2.0 * (double)G[8 * plane + x]);
    q_out += ((double)G[4 * plane + top + x] + (double)G[7 * plane + top + x] + (double)G[8 * plane + top + x]) -
             ((double)G[2 * plane + top + x] + (double)G[5 * plane + top + x] + (double)G[6 * plane + top + x]);
  }
  q_in = block_sum(q_in, red);
  q_out = block_sum(q_out, red);
  double v[7] = {0, 0, 0, 0, 0, -1e300, 0};
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    for (int q = 0; q < 4; ++q) v[q] += part[8 * b + q];
    for (int q = 4; q < 7; ++q) v[q] = fmax(v[q], part[8 * b + q]);
  }
  for (int q = 0; q < 4; ++q) v[q] = block_sum(v[q], red);
  for (int q = 4; q < 7; ++q) v[q] = block_max(v[q], red);
  if (threadIdx.x == 0) {
    const double n = (double)c.ny * c.nx;
    out[1] = v[0];
    out[2] = v[1];
    out[3] = sqrt(v[2] / n);
    out[4] = v[4];
    out[5] = -v[5];
    out[6] = v[3];
    out[7] = v[6];
    out[8] = q_in;
    out[9] = q_out;
  }
}

// ------------------------------------------------------ batched kernels
// One launch per kernel type covers every slot of a batch; each block finds
// its slot from the per-launch block offsets.

// The last slot s < ns with off[s] <= b (offsets non-decreasing, off[0] =
// 0; slots without blocks share their offset with the next one).  Every
// wave compares 64 offsets at once and counts them with a ballot: one load
// for ns <= 64, two (every 64th offset, then 64 of them) up to 4096 slots,
// instead of a chain of dependent loads.  Called with all lanes active.
__device__ __forceinline__ int find_slot(const int* __restrict__ off, int ns, int b) {
  const int lane = threadIdx.x & 63;
  int base = 0;
  if (ns > 64) {
    const int i = lane * 64;
    base = 64 * (__popcll(__ballot(i < ns && off[i] <= b)) - 1);
  }
  const int i = base + lane;
  return base + __popcll(__ballot(i < ns && off[i] <= b)) - 1;
}

// Threads per block of the batched chunk solves: one wave, so that the few
// (m, chunk) threads of small instances spread over more CUs.
constexpr int kBatchTriThreads = 64;

__device__ __forceinline__ bool slot_emits(const SlotDesc& d) {
  const long long k = d.steps_done + 1;  // the step being taken
  return k == d.steps_target || (d.emit_every > 0 && k % d.emit_every == 0);
}

template <typename T, int F>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(TransformWaves<T, F>::value))) kb_forward(const SlotDesc* __restrict__ D, const int* __restrict__ off, int ns) {
  const int s = find_slot(off, ns, blockIdx.x);
  const SlotDesc& d = D[s];
  if (!d.active) return;
  const ChargeSrc<T> q{(const T*)d.b.rq, (const T*)d.b.eu, (const T*)d.b.ed, nullptr, nullptr};
  forward_body<T, 0, F>(d.c, q, d.plan, (const C2<T>*)d.b.tw, (C2<T>*)d.b.spec, d.b.rowsd + ROWD_DCSUM * d.c.ny,
                     blockIdx.x - off[s]);
}

template <typename T>
__global__ void __launch_bounds__(256) kb_tri_local(const SlotDesc* __restrict__ D, const int* __restrict__ off,
                                                    int ns) {
  const int s = find_slot(off, ns, blockIdx.x);
  const SlotDesc& d = D[s];
  if (!d.active) return;
  const int lb = blockIdx.x - off[s];
  const int nbx = (d.c.M - 1 + blockDim.x - 1) / blockDim.x;
  tri_local_body<T>(d.c, (const T*)d.b.tt, (C2<T>*)d.b.spec, (C2<T>*)d.b.ends, lb % nbx, lb / nbx);
}

// 256 threads per block: four wavenumbers per block on the scan path, 256 on
// the serial one (chosen per slot by its interface count).
template <typename T>
__global__ void __launch_bounds__(256) kb_tri_reduced(const SlotDesc* __restrict__ D, const int* __restrict__ off,
                                                      int ns) {
  const int s = find_slot(off, ns, blockIdx.x);
  const SlotDesc& d = D[s];
  if (!d.active) return;
  const int lb = blockIdx.x - off[s];
  if (d.c.NC - 1 <= kScanMax) {
    const int m = 1 + lb * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (m >= d.c.M) return;
    tri_scan_body<T>(d.c, (const T*)d.b.rf, (const C2<T>*)d.b.ends, (C2<T>*)d.b.iface, m);
  } else {
    tri_reduced_body<T>(d.c, (const T*)d.b.tt, (const C2<T>*)d.b.ends, (T*)d.b.gh, (C2<T>*)d.b.iface, lb);
  }
}

template <typename T, int F>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(TransformWaves<T, F>::value))) kb_inverse(const SlotDesc* __restrict__ D, const int* __restrict__ off, int ns) {
  const int s = find_slot(off, ns, blockIdx.x);
  const SlotDesc& d = D[s];
  if (!d.active) return;
  const int lb = blockIdx.x - off[s];
  if (lb == 0) {
    mean_mode_body(d.c, d.b.rowsd, d.b.dmean);
    return;
  }
  inverse_body<T, F>(d.c, (const C2<T>*)d.b.spec, (const T*)d.b.tt, (const C2<T>*)d.b.iface, d.plan,
                     (const C2<T>*)d.b.tw, (T*)d.b.phi, lb - 1);
}

template <typename T, typename C>
__global__ void __launch_bounds__(1024) kb_collide(const SlotDesc* __restrict__ D, const int* __restrict__ off,
                                                   int ns) {
  const int s = find_slot(off, ns, blockIdx.x);
  const SlotDesc& d = D[s];
  if (!d.active) return;
  const int src = d.cur, dst = 1 - d.cur;
  const int b = blockIdx.x - off[s];
  if (slot_emits(d))
    collide_tile<T, C, true, true>(d.c, (const T*)d.b.f[src], (const T*)d.b.g[src], (T*)d.b.f[dst],
                                   (T*)d.b.g[dst], (const T*)d.b.phi, (const T*)d.b.rows, d.b.rowsd, d.b.mom,
                                   (T*)d.b.rq, (T*)d.b.eu, (T*)d.b.ed, b);
  else
    collide_tile<T, C, true, false>(d.c, (const T*)d.b.f[src], (const T*)d.b.g[src], (T*)d.b.f[dst],
                                    (T*)d.b.g[dst], (const T*)d.b.phi, (const T*)d.b.rows, d.b.rowsd, d.b.mom,
                                    (T*)d.b.rq, (T*)d.b.eu, (T*)d.b.ed, b);
}
// End of a batched step, one block per slot: the diagnostics of a slot that
// emitted moments this step (into its history), then the device-side advance of every active slot (flip the
// buffers, count the step, retire the slot at its target), so a captured
// multi-step graph needs no host updates.
template <typename T>
__global__ void __launch_bounds__(256) kb_stats_advance(SlotDesc* __restrict__ D, const int* __restrict__ off,
                                                        int ns) {
  __shared__ double red[16];
  const int s = find_slot(off, ns, blockIdx.x);
  SlotDesc& d = D[s];
  if (!d.active) return;
  const long long k = d.steps_done + 1;  // the step just taken
  if (slot_emits(d) && d.hist != nullptr) {
    const int row = (d.emit_every > 0 && k % d.emit_every == 0) ? (int)(k / d.emit_every) - 1 : d.hist_cap - 1;
    if (row >= 0 && row < d.hist_cap) {
      const int nx = d.c.nx, ny = d.c.ny;
      const size_t n = (size_t)ny * nx;
      // a1: the largest over the rows of |sum_x u_y exp(-2 pi i x / nx)| / nx,
      // the amplitude of the first x mode (the perturbation whose growth or
      // decay marks the electroconvective threshold).  Rows go to the waves
      // in turn; a wave reduces its row's mode with shuffles, the block then
      // reduces the per-lane sums and maxima (fixed order for a fixed block
      // size).
      const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
      double suy = 0, srho_c = 0, mu = 0, a1 = 0, bad = 0;
      for (int j = wave; j < ny; j += nw) {
        const double r = d.b.rowsd[ROWD_R * ny + j], rr = d.b.rowsd[ROWD_RHO_REF * ny + j];
        double cr = 0, ci = 0;
        for (int x = lane; x < nx; x += 64) {
          const size_t q = (size_t)j * nx + x;
          const double ux = d.b.mom[n + q], uy = d.b.mom[2 * n + q];
          const double rho = rr + d.b.mom[q], rc = r + d.b.mom[3 * n + q];
          suy += uy * uy;
          mu = fmax(mu, sqrt(ux * ux + uy * uy));
          srho_c += rc;
          if (!(rho > 0.0) || !isfinite(rho) || !isfinite(ux) || !isfinite(uy) || !isfinite(rc)) bad += 1.0;
          double sn, cs;
          sincospi(2.0 * (double)x / (double)nx, &sn, &cs);
          cr += uy * cs;
          ci -= uy * sn;
        }
        cr = wave_sum(cr);
        ci = wave_sum(ci);
        a1 = fmax(a1, sqrt(cr * cr + ci * ci) / (double)nx);
      }
      // collector current: what leaves through the upper electrode in the
      // next streaming, from the post-collision populations just written
      // (the reference rows cancel between the up and the down directions;
      // a whole-row sum, so the x shift of the stored movers does not matter)
      const T* G = (const T*)d.b.g[1 - d.cur];
      const size_t plane = (size_t)ny * d.c.P, top = (size_t)(ny - 1) * d.c.P;
      double cur_out = 0;
      for (int x = threadIdx.x; x < nx; x += blockDim.x)
        cur_out += ((double)G[2 * plane + top + x] + (double)G[5 * plane + top + x] +
                    (double)G[6 * plane + top + x]) -
                   ((double)G[4 * plane + top + x] + (double)G[7 * plane + top + x] +
                    (double)G[8 * plane + top + x]);
      cur_out = block_sum(cur_out, red);
      suy = block_sum(suy, red);
      srho_c = block_sum(srho_c, red);
      mu = block_max(mu, red);
      a1 = block_max(a1, red);
      bad = block_sum(bad, red);
      if (threadIdx.x == 0) {
        double* h = d.hist + kHistCols * (size_t)row;
        h[0] = (double)k;
        h[1] = sqrt(suy / (double)n);
        h[2] = mu;
        h[3] = srho_c;
        h[4] = a1;
        h[5] = bad;
        h[6] = cur_out;
      }
    }
  }
  __syncthreads();  // every thread has read the step state
  if (threadIdx.x == 0) {
    d.cur = 1 - d.cur;
    d.steps_done = k;
    if (k >= d.steps_target) d.active = 0;
  }
}

int batch_blocks(const Consts& c, int k) {
  const int nm = c.M - 1;
  switch (k) {
    case BK_FORWARD: return (c.ny + 1) / 2;
    case BK_INVERSE: return 1 + (c.ny + 1) / 2;  // block 0: the x-mean mode
    case BK_TRI_LOCAL: return nm > 0 ? ((nm + kBatchTriThreads - 1) / kBatchTriThreads) * c.NC : 0;
    case BK_TRI_REDUCED:
      if (nm <= 0 || c.NC < 2) return 0;
      return c.NC - 1 <= kScanMax ? (nm + 3) / 4 : (nm + 255) / 256;
    case BK_COLLIDE: return collide_blocks(c);
    case BK_STATS: return 1;
  }
  return 0;
}

template <typename T, typename C>
hipError_t launch_batch_step(const SlotDesc* d_desc, const int* d_off, const int* totals, int ns, size_t lds,
                             size_t collide_lds, bool fft8, const Tuning& tu, hipStream_t s) {
  const int row = ns + 1;
  SlotDesc* D = const_cast<SlotDesc*>(d_desc);
  if (totals[BK_FORWARD]) {
    if (fft8)
      hipLaunchKernelGGL((kb_forward<T, 8>), dim3(totals[BK_FORWARD]), dim3(tu.fft_threads), lds, s, d_desc,
                         d_off + BK_FORWARD * row, ns);
    else
      hipLaunchKernelGGL((kb_forward<T, kFftPerThread>), dim3(totals[BK_FORWARD]), dim3(tu.fft_threads), lds, s,
                         d_desc, d_off + BK_FORWARD * row, ns);
  }
  if (totals[BK_TRI_LOCAL])
    hipLaunchKernelGGL(kb_tri_local<T>, dim3(totals[BK_TRI_LOCAL]), dim3(kBatchTriThreads), 0, s, d_desc,
                       d_off + BK_TRI_LOCAL * row, ns);
  if (totals[BK_TRI_REDUCED])
    hipLaunchKernelGGL(kb_tri_reduced<T>, dim3(totals[BK_TRI_REDUCED]), dim3(256), 0, s, d_desc,
                       d_off + BK_TRI_REDUCED * row, ns);
  if (totals[BK_INVERSE]) {
    if (fft8)
      hipLaunchKernelGGL((kb_inverse<T, 8>), dim3(totals[BK_INVERSE]), dim3(tu.fft_threads), lds, s, d_desc,
                         d_off + BK_INVERSE * row, ns);
    else
      hipLaunchKernelGGL((kb_inverse<T, kFftPerThread>), dim3(totals[BK_INVERSE]), dim3(tu.fft_threads), lds, s,
                         d_desc, d_off + BK_INVERSE * row, ns);
  }
  if (totals[BK_COLLIDE])
    hipLaunchKernelGGL((kb_collide<T, C>), dim3(totals[BK_COLLIDE]), dim3(tu.cbx * tu.cby), collide_lds, s, d_desc,
                       d_off + BK_COLLIDE * row, ns);
  if (totals[BK_STATS])
    hipLaunchKernelGGL(kb_stats_advance<T>, dim3(totals[BK_STATS]), dim3(256), 0, s, D, d_off + BK_STATS * row, ns);
  return hipGetLastError();
}

template hipError_t launch_batch_step<double, double>(const SlotDesc*, const int*, const int*, int, size_t, size_t, bool,
                                                     const Tuning&, hipStream_t);
template hipError_t launch_batch_step<float, float>(const SlotDesc*, const int*, const int*, int, size_t, size_t, bool,
                                                   const Tuning&, hipStream_t);
template hipError_t launch_batch_step<float, double>(const SlotDesc*, const int*, const int*, int, size_t, size_t, bool,
                                                    const Tuning&, hipStream_t);

// ------------------------------------------------------------- launchers
template <typename T>
hipError_t launch_init_charge(const Consts& c, const Bufs& b, hipStream_t s) {
  dim3 blk(256), grd((c.nx + 255) / 256, c.ny);
  hipLaunchKernelGGL(k_init_charge<T>, grd, blk, 0, s, c, b.rowsd, b.mom);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_init_populations(const Consts& c, const Bufs& b, int dst, hipStream_t s) {
  dim3 blk(256), grd((c.nx + 255) / 256, c.ny);
  hipLaunchKernelGGL(k_init_populations<T>, grd, blk, 0, s, c, (T*)b.f[dst], (T*)b.g[dst], (const T*)b.phi,
                     b.rowsd, b.mom);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_forward(const Consts& c, const Bufs& b, const FftPlan& pl, int mode, int src, const Tuning& tu,
                          hipStream_t s) {
  dim3 blk(tu.fft_threads), grd((c.ny + 1) / 2);
  const size_t lds = fft_lds_bytes<T>(pl, tu.fft_threads);
  const ChargeSrc<T> q{(const T*)b.rq, (const T*)b.eu, (const T*)b.ed, (const T*)b.g[src],
                       b.mom + 3 * (size_t)c.ny * c.nx};
  C2<T>* spec = (C2<T>*)b.spec;
  const C2<T>* tw = (const C2<T>*)b.tw;
  double* dcs = b.rowsd + ROWD_DCSUM * c.ny;
  const bool f8 = fft_in_place(pl, tu.fft_threads, 8);
  if (mode == 0 && f8)
    hipLaunchKernelGGL((k_forward<T, 0, 8>), grd, blk, lds, s, c, q, pl, tw, spec, dcs);
  else if (mode == 0)
    hipLaunchKernelGGL((k_forward<T, 0, kFftPerThread>), grd, blk, lds, s, c, q, pl, tw, spec, dcs);
  else if (mode == 1)
    hipLaunchKernelGGL((k_forward<T, 1, kFftPerThread>), grd, blk, lds, s, c, q, pl, tw, spec, dcs);
  else
    hipLaunchKernelGGL((k_forward<T, 2, kFftPerThread>), grd, blk, lds, s, c, q, pl, tw, spec, dcs);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tridiag(const Consts& c, const Bufs& b, hipStream_t s) {
  const int nm = c.M - 1;
  if (nm <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tri_local<T>, dim3(((nm + 255) / 256) * c.NC), dim3(256), 0, s, c, (const T*)b.tt,
                     (C2<T>*)b.spec, (C2<T>*)b.ends);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || c.NC < 2) return e;
  if (c.NC - 1 <= kScanMax)
    hipLaunchKernelGGL(k_tri_scan<T>, dim3((nm + 3) / 4), dim3(256), 0, s, c, (const T*)b.rf,
                       (const C2<T>*)b.ends, (C2<T>*)b.iface);
  else
    hipLaunchKernelGGL(k_tri_reduced<T>, dim3((nm + 63) / 64), dim3(64), 0, s, c, (const T*)b.tt,
                       (const C2<T>*)b.ends, (T*)b.gh, (C2<T>*)b.iface);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_inverse(const Consts& c, const Bufs& b, const FftPlan& pl, const Tuning& tu, hipStream_t s) {
  dim3 blk(tu.fft_threads), grd(1 + (c.ny + 1) / 2);  // block 0: the x-mean mode
  const size_t lds = fft_lds_bytes<T>(pl, tu.fft_threads);
  if (fft_in_place(pl, tu.fft_threads, 8))
    hipLaunchKernelGGL((k_inverse<T, 8>), grd, blk, lds, s, c, (const C2<T>*)b.spec, (const T*)b.tt,
                       (const C2<T>*)b.iface, pl, (const C2<T>*)b.tw, (T*)b.phi, b.rowsd, b.dmean);
  else
    hipLaunchKernelGGL((k_inverse<T, kFftPerThread>), grd, blk, lds, s, c, (const C2<T>*)b.spec, (const T*)b.tt,
                       (const C2<T>*)b.iface, pl, (const C2<T>*)b.tw, (T*)b.phi, b.rowsd, b.dmean);
  return hipGetLastError();
}

template <typename T, typename C>
hipError_t launch_collide(const Consts& c0, const Bufs& b, bool pull, bool emit, int src, int dst,
                          const Tuning& tu, hipStream_t s) {
  Consts c = c0;
  c.TW = tile_width(c.nx, tu.ctw, (int)sizeof(T));
  dim3 blk(tu.cbx * tu.cby), grd(collide_blocks(c));
  const size_t lds = collide_lds_bytes<T>(c.TW, c.nx);
  const T* Fin = (const T*)b.f[src];
  const T* Gin = (const T*)b.g[src];
  T* Fout = (T*)b.f[dst];
  T* Gout = (T*)b.g[dst];
  const T* phi = (const T*)b.phi;
  const T* rows = (const T*)b.rows;
  T* rq = (T*)b.rq;
  T* eu = (T*)b.eu;
  T* ed = (T*)b.ed;
  if (pull && emit)
    hipLaunchKernelGGL((k_collide<T, C, true, true>), grd, blk, lds, s, c, Fin, Gin, Fout, Gout, phi, rows, b.rowsd,
                       b.mom, rq, eu, ed);
  else if (pull)
    hipLaunchKernelGGL((k_collide<T, C, true, false>), grd, blk, lds, s, c, Fin, Gin, Fout, Gout, phi, rows,
                       b.rowsd, b.mom, rq, eu, ed);
  else if (emit)
    hipLaunchKernelGGL((k_collide<T, C, false, true>), grd, blk, lds, s, c, Fin, Gin, Fout, Gout, phi, rows,
                       b.rowsd, b.mom, rq, eu, ed);
  else
    hipLaunchKernelGGL((k_collide<T, C, false, false>), grd, blk, lds, s, c, Fin, Gin, Fout, Gout, phi, rows,
                       b.rowsd, b.mom, rq, eu, ed);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fields(const Consts& c, const Bufs& b, double* rho, double* ux, double* uy, double* rho_c,
                         double* phi, double* rho_m1, hipStream_t s) {
  dim3 blk(256), grd((c.nx + 255) / 256, c.ny);
  hipLaunchKernelGGL(k_fields<T>, grd, blk, 0, s, c, b.mom, (const T*)b.phi, b.rowsd, rho, ux, uy, rho_c, phi,
                     rho_m1);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_charge_in(const Consts& c, const Bufs& b, const double* rho_c_nd, hipStream_t s) {
  dim3 blk(256), grd((c.nx + 255) / 256, c.ny);
  hipLaunchKernelGGL(k_charge_in, grd, blk, 0, s, c, rho_c_nd, b.rowsd, b.mom);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_stats(const Consts& c, const Bufs& b, int cur, hipStream_t s) {
  const int nb = c.ny < kStatsBands ? c.ny : kStatsBands;
  hipLaunchKernelGGL(k_stats_part<T>, dim3(nb), dim3(256), 0, s, c, b.mom, (const T*)b.phi, b.rowsd, b.spart);
  hipLaunchKernelGGL(k_stats_final<T>, dim3(1), dim3(256), 0, s, c, (const double*)b.spart, nb,
                     (const T*)b.g[cur], b.stats);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_continue(const Consts& c, const Bufs& b, int cur, double scale, double ddelta, hipStream_t s) {
  dim3 blk(256), grd((c.nx + 255) / 256, c.ny);
  hipLaunchKernelGGL(k_continue<T>, grd, blk, 0, s, c, (T*)b.f[cur], (T*)b.g[cur], b.mom, b.rowsd, scale, ddelta);
  return hipGetLastError();
}

template <typename T>
size_t yspec_lds_bytes(int ny) {
  return 2 * (size_t)(2 * ny) * sizeof(C2<T>);
}

template <typename T>
hipError_t launch_yspec(const Consts& c, const Bufs& b, const FftPlan& py, hipStream_t s) {
  if (c.M < 2) return hipSuccess;  // no m >= 1 modes
  if (fft_in_place(py, 512, kFftPerThread))
    hipLaunchKernelGGL(k_yspec_ip<T>, dim3(c.M - 1), dim3(512), (size_t)py.n * sizeof(C2<T>), s, c, py,
                       (const C2<T>*)b.twy, (C2<T>*)b.spec);
  else
    hipLaunchKernelGGL(k_yspec<T>, dim3(c.M - 1), dim3(256), yspec_lds_bytes<T>(c.ny), s, c, py,
                       (const C2<T>*)b.twy, (C2<T>*)b.spec);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_density(const Consts& c0, const Bufs& b, int cur, const Tuning& tu, hipStream_t s) {
  Consts c = c0;
  c.TW = tile_width(c.nx, tu.ctw, (int)sizeof(T));
  hipLaunchKernelGGL(k_density<T>, dim3(collide_blocks(c)), dim3(tu.cbx * tu.cby), collide_lds_bytes<T>(c.TW, c.nx), s, c,
                     (const T*)b.g[cur], (const T*)b.rows, (T*)b.rq, (T*)b.eu, (T*)b.ed);
  return hipGetLastError();
}

#define EC_INSTANTIATE(T)                                                                                   \
  template hipError_t launch_init_charge<T>(const Consts&, const Bufs&, hipStream_t);                       \
  template hipError_t launch_init_populations<T>(const Consts&, const Bufs&, int, hipStream_t);             \
  template hipError_t launch_forward<T>(const Consts&, const Bufs&, const FftPlan&, int, int, const Tuning&,   \
                                       hipStream_t);                                                        \
  template hipError_t launch_tridiag<T>(const Consts&, const Bufs&, hipStream_t);                           \
  template hipError_t launch_inverse<T>(const Consts&, const Bufs&, const FftPlan&, const Tuning&, hipStream_t); \
  template hipError_t launch_fields<T>(const Consts&, const Bufs&, double*, double*, double*, double*,       \
                                       double*, double*, hipStream_t);                                      \
  template hipError_t launch_charge_in<T>(const Consts&, const Bufs&, const double*, hipStream_t);          \
  template hipError_t launch_stats<T>(const Consts&, const Bufs&, int, hipStream_t);                        \
  template hipError_t launch_continue<T>(const Consts&, const Bufs&, int, double, double, hipStream_t);     \
  template hipError_t launch_density<T>(const Consts&, const Bufs&, int, const Tuning&, hipStream_t);         \
  template hipError_t launch_yspec<T>(const Consts&, const Bufs&, const FftPlan&, hipStream_t);              \
  template size_t yspec_lds_bytes<T>(int);

EC_INSTANTIATE(double)
EC_INSTANTIATE(float)
template hipError_t launch_collide<double, double>(const Consts&, const Bufs&, bool, bool, int, int, const Tuning&,
                                                  hipStream_t);
template hipError_t launch_collide<float, float>(const Consts&, const Bufs&, bool, bool, int, int, const Tuning&,
                                                hipStream_t);
template hipError_t launch_collide<float, double>(const Consts&, const Bufs&, bool, bool, int, int, const Tuning&,
                                                 hipStream_t);

}  // namespace ec
