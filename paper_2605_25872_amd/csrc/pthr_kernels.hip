// PTHR kernels for gfx950 (CDNA4).
//
// One workgroup owns one disorder sample for the whole launch.  Its LDS holds
// every clone's spins bit-packed 32 clones per word: word w of site j is a
// 32-bit mask whose bit b is clone 32w+b (1 = spin down).  Sites are split by
// checkerboard colour, j = colour*V/2 + i/2, so the sites one colour updates
// are contiguous and their neighbours are all in the other half.  Each
// work-item owns `CH` consecutive natural sites (CH/2 of each colour) and keeps
// their six couplings in registers for the whole launch; one 32-bit LDS load of
// a neighbour word serves the 32 clones that share that site and those
// couplings (the paper's multispin idea, App. A.1, carried to 32 clones per
// word).  Each phase of an elementary Monte Carlo step (paper Sec. 3) is its
// own kernel: it loads the sample into LDS, runs, and writes back.
//
// Exactness: every random number is a Philox4x32-10 block keyed by
// (seed; site | sweep<<16 | purpose<<24, EMCS, slot, sample), and every
// floating-point result is produced by a fixed sequence of correctly rounded
// operations (explicit fma, no contraction), so any launch shape gives the
// same bits.

#include <hip/hip_runtime.h>

#include <type_traits>

#include "pthr_internal.h"

namespace pthr {
namespace {

constexpr int kWave = 64;
constexpr int kMaxThreads = 1024;
constexpr int kMaxWaves = kMaxThreads / kWave;

// ---------------------------------------------------------------- random bits
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
struct Block {
  uint32_t w0, w1, w2, w3;
};
// float(w) of a block's four words (the FP32 Metropolis and heat-bath tests
// use them); converted as soon as the block is taken up, so that its integer
// words are dead before the next block is produced
struct Floats4 {
  float u[4];
};
__device__ __forceinline__ Floats4 to_floats(const Block& b) {
  return {{static_cast<float>(b.w0), static_cast<float>(b.w1), static_cast<float>(b.w2), static_cast<float>(b.w3)}};
}
// FP64 tests: the float of the 53 random bits of each word pair (u[0]: w0,
// w1; u[1]: w2, w3), formed as bits53 does.
__device__ __forceinline__ Floats4 to_bits53(const Block& b) {
  return {{__builtin_fmaf(static_cast<float>(b.w1), 0x1p21f, static_cast<float>(b.w0 >> 11)),
           __builtin_fmaf(static_cast<float>(b.w3), 0x1p21f, static_cast<float>(b.w2 >> 11)), 0.0f, 0.0f}};
}

// a ^ b ^ k in one VALU operation (three-input bitwise function, truth table
// 0x96); k is wave-uniform and read from a scalar register.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t k) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
  return r;
}

__device__ __forceinline__ Block philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t pa = static_cast<uint64_t>(0xD2511F53u) * c0;
    const uint64_t pb = static_cast<uint64_t>(0xCD9E8D57u) * c2;
    uint32_t n0, n2;
    // The first rounds often see wave-uniform counter words: their XORs are
    // left to the compiler, which keeps uniform parts on the scalar unit.
    if (round < 2) {
      n0 = static_cast<uint32_t>(pb >> 32) ^ c1 ^ k0;
    } else {
      n0 = xor3(static_cast<uint32_t>(pb >> 32), c1, k0);
    }
    if (round < 3) {
      n2 = static_cast<uint32_t>(pa >> 32) ^ c3 ^ k1;
    } else {
      n2 = xor3(static_cast<uint32_t>(pa >> 32), c3, k1);
    }
    c1 = static_cast<uint32_t>(pb);
    c3 = static_cast<uint32_t>(pa);
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Block{c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t ctr_word(uint32_t site, uint32_t m, uint32_t purpose) {
  return site | (m << 16) | (purpose << 24);
}

// [0,1) with 53 random bits: exact.
__device__ __forceinline__ double uniform53(uint32_t lo, uint32_t hi) {
  const uint64_t bits = ((static_cast<uint64_t>(hi) << 32) | lo) >> 11;
  return static_cast<double>(bits) * 0x1p-53;
}
// [0,1] from one word rounded to float (FP32 form).
__device__ __forceinline__ float uniform32(uint32_t w) {
  return static_cast<float>(w) * 0x1p-32f;
}

// ---------------------------------------------------------------- exp(x), x <= 0
// Cody-Waite: x = k ln2 + r with ln2 split in a 32-bit head and a tail, then
// sum_{n<=13} r^n/n! by Horner with fused multiply-adds (1/n! rounded to
// double), scaled by 2^k.  The result lies strictly inside (2^(k-1), 2^(k+1)).
__device__ __forceinline__ double exp_poly64(double x, double k) {
  double r = __builtin_fma(-k, 0x1.62e42feep-1, x);
  r = __builtin_fma(-k, 0x1.a39ef35793c76p-33, r);
  double p = 0x1.6124613a86d09p-33;             // 1/13!
  p = __builtin_fma(p, r, 0x1.1eed8eff8d898p-29); // 1/12!
  p = __builtin_fma(p, r, 0x1.ae64567f544e4p-26); // 1/11!
  p = __builtin_fma(p, r, 0x1.27e4fb7789f5cp-22); // 1/10!
  p = __builtin_fma(p, r, 0x1.71de3a556c734p-19); // 1/9!
  p = __builtin_fma(p, r, 0x1.a01a01a01a01ap-16); // 1/8!
  p = __builtin_fma(p, r, 0x1.a01a01a01a01ap-13); // 1/7!
  p = __builtin_fma(p, r, 0x1.6c16c16c16c17p-10); // 1/6!
  p = __builtin_fma(p, r, 0x1.1111111111111p-7);  // 1/5!
  p = __builtin_fma(p, r, 0x1.5555555555555p-5);  // 1/4!
  p = __builtin_fma(p, r, 0x1.5555555555555p-3);  // 1/3!
  p = __builtin_fma(p, r, 0x1p-1);                // 1/2!
  p = __builtin_fma(p, r, 1.0);                   // 1/1!
  p = __builtin_fma(p, r, 1.0);                   // 1/0!
  return __builtin_ldexp(p, static_cast<int>(k));
}
__device__ __forceinline__ double exp_neg64(double x) {
  if (x < -708.0) return 0.0;
  return exp_poly64(x, __builtin_rint(x * 0x1.71547652b82fep+0));
}

// FP32 form, in base 2: 2^t for t = -(beta log2 e) dE.  t = k + f with
// k = rint(t) and f = t - k (exact, |f| <= 1/2); 2^f by the degree-6
// polynomial 1 + c1 f + ... + c6 f^6 whose coefficients (rounded to float)
// minimise the largest relative error on |f| <= 1/2 (within 0.952 float ulp
// of 2^f for every float f there), Horner with fused multiply-adds, then 2^k.
// The result lies strictly inside (2^(k-1), 2^(k+1)).
__device__ __forceinline__ float exp2_frac32(float f) {
  float p = 0x1.41fbbcp-13f;
  p = __builtin_fmaf(p, f, 0x1.5f3e54p-10f);
  p = __builtin_fmaf(p, f, 0x1.3b2d4cp-7f);
  p = __builtin_fmaf(p, f, 0x1.c6aee8p-5f);
  p = __builtin_fmaf(p, f, 0x1.ebfbdcp-3f);
  p = __builtin_fmaf(p, f, 0x1.62e430p-1f);
  return __builtin_fmaf(p, f, 1.0f);
}
__device__ __forceinline__ float exp2_poly32(float f, float k) {
  return __builtin_ldexpf(exp2_frac32(f), static_cast<int>(k));
}
// 2^t * 2^32 with the same rounding steps as exp2_poly32: every Horner
// coefficient is scaled by 2^32, which commutes with each rounding (the
// polynomial stays far from overflow and underflow), so float(w) <=
// exp2_poly32_x2p32(f, k) decides exactly as float(w) * 2^-32 <=
// exp2_poly32(f, k) (where the scaled 2^k underflows, float(w) * 2^-32 is 0
// or at least 2^-32 and both sides agree).
// exp2_frac32's coefficients c0 .. c6 scaled by 2^32.
constexpr float kExp2x2p32[7] = {0x1p+32f,       0x1.62e430p+31f, 0x1.ebfbdcp+29f, 0x1.c6aee8p+27f,
                                 0x1.3b2d4cp+25f, 0x1.5f3e54p+22f, 0x1.41fbbcp+19f};
__device__ __forceinline__ float exp2_poly32_x2p32(float f, int k) {
  float p = kExp2x2p32[6];
#pragma unroll
  for (int n = 5; n >= 0; --n) p = __builtin_fmaf(p, f, kExp2x2p32[n]);
  return __builtin_ldexpf(p, k);
}

// (a & mask) | (b & ~mask) as one v_bfi_b32.
__device__ __forceinline__ uint32_t bitfield_insert(uint32_t mask, uint32_t a, uint32_t b) {
  uint32_t r;
  asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(mask), "v"(a), "v"(b));
  return r;
}

// (f << 1) | bit, bit = this lane's bit of the wave mask `lanes`, as one
// v_addc_co_u32 (f + f + carry-in).
__device__ __forceinline__ uint32_t shift_in(uint32_t f, uint64_t lanes) {
  uint32_t r;
  uint64_t carry_out;
  asm("v_addc_co_u32_e64 %0, %1, %2, %2, %3" : "=v"(r), "=s"(carry_out) : "v"(f), "s"(lanes));
  return r;
}

// Metropolis test for dE > 0: FP64 "u < exp(x)", x = -beta dE; FP32
// "u <= 2^t", t = -(beta log2 e) dE.  With `early` the binade bracket
// 2^(k-1) < value < 2^(k+1) decides it without the polynomial unless u falls
// inside the bracket; both forms return the same decision.
// flip_sign(v, s) is v with its sign flipped where bit 31 of s is set.
template <typename FP>
struct Prec;
template <>
struct Prec<double> {
  static __device__ __forceinline__ double u(const Block& b, int word_pair) {
    return word_pair ? uniform53(b.w2, b.w3) : uniform53(b.w0, b.w1);
  }
  static __device__ __forceinline__ bool accept(double u, double x, bool early) {
    if (x < -708.0) return false;
    const double k = __builtin_rint(x * 0x1.71547652b82fep+0);
    if (early) {
      const int ki = static_cast<int>(k);
      if (u < __builtin_ldexp(1.0, ki - 1)) return true;
      if (!(u < __builtin_ldexp(1.0, ki + 1))) return false;
    }
    return u < exp_poly64(x, k);
  }
  // Same decision as accept(u, x, false) for x <= 0, as a mask over the
  // wave's lanes.  With x = k ln2 + r (the reduction of exp_poly64), the test
  // u < p 2^k is d < p for d = u 2^-k (exact scaling for these u and k), p
  // the FP64 polynomial's value of e^r.  It is first decided against
  // q = exp2_frac32(float(r) log2 e), within 1.3e-7 of e^r relative (at most
  // 1.05e-7 for every float r with |r| <= 0.35, checked exhaustively, plus
  // the rounding of r to float): d in float below q (1 - 2^-20) proves
  // acceptance and at or above q (1 + 2^-20) proves rejection, the roundings
  // of d (2^-23) and of the two bounds (2^-24 each) included.
  // Only when some lane falls between the bounds (about once in 10^6 tests)
  // does the wave evaluate the FP64 polynomial (the caller redoes the word).
  // u is uniform53(lo, hi); bound factors f_lo = 1 - 2^-20 and
  // f_hi = 1 + 2^-20 (with 0 and +inf every lane is left open).
  struct Bound {
    uint64_t sure;  // lanes whose test the bound proves accepted
    uint64_t open;  // lanes in range the bound leaves undecided
  };
  // The 53 random bits hi 2^21 + (lo >> 11) of u = (bits) 2^-53 in float:
  // float(hi) and the fused multiply-add round once each (the low part is
  // exact), so the result is within 2^-23 of the bits, relative.
  static __device__ __forceinline__ float bits53(uint32_t lo, uint32_t hi) {
    return __builtin_fmaf(static_cast<float>(hi), 0x1p21f, static_cast<float>(lo >> 11));
  }
  // hb: bits53 of the test's random words.
  static __device__ __forceinline__ Bound bound_lanes(float hb, double x, float f_lo, float f_hi) {
    const double k = __builtin_rint(x * 0x1.71547652b82fep+0);
    double r = __builtin_fma(-k, 0x1.62e42feep-1, x);
    r = __builtin_fma(-k, 0x1.a39ef35793c76p-33, r);
    const float q = exp2_frac32(static_cast<float>(r) * 0x1.715476p+0f);
    // u 2^-k in float: d is within 2^-23 of u 2^-k relative (or is 0 or
    // subnormal where u 2^-k is far below q, or +inf where it is far above)
    const float d = __builtin_ldexpf(hb, -53 - static_cast<int>(k));
    const uint64_t in_range = __builtin_amdgcn_ballot_w64(x >= -708.0);
    const uint64_t below = __builtin_amdgcn_ballot_w64(d < q * f_lo);
    const uint64_t above = __builtin_amdgcn_ballot_w64(!(d < q * f_hi));
    return Bound{in_range & below, in_range & ~below & ~above};
  }
  // The test with the FP64 polynomial for every lane (k = rint(x log2 e)).
  static __device__ __forceinline__ uint64_t exact_lanes(uint32_t lo, uint32_t hi, double x, double k) {
    return __builtin_amdgcn_ballot_w64(x >= -708.0) & __builtin_amdgcn_ballot_w64(uniform53(lo, hi) < exp_poly64(x, k));
  }
  // Heat bath: flip with probability 1 / (1 + exp(beta dE)), tested as
  // fma(u, a, u) < (dE > 0 ? a : 1) with a = exp(-beta |dE|) (0 below -708).
  static __device__ __forceinline__ uint64_t heat_bath_lanes(double u, double beta, double dE) {
    const double x = -(beta * __builtin_fabs(dE));
    const double p = exp_poly64(x, __builtin_rint(x * 0x1.71547652b82fep+0));
    const double a = x >= -708.0 ? p : 0.0;
    return __builtin_amdgcn_ballot_w64(__builtin_fma(u, a, u) < (dE > 0.0 ? a : 1.0));
  }
  static __device__ __forceinline__ double flip_sign(double v, uint32_t s) {
    return __hiloint2double(static_cast<int>((s & 0x80000000u) ^ static_cast<uint32_t>(__double2hiint(v))),
                            __double2loint(v));
  }
};
template <>
struct Prec<float> {
  // FP32 form: x is t = -(beta log2 e) dE; accept iff u <= 2^t (every
  // dE <= 0 passes; 2^t overflows to +inf and underflows to 0, and u is 0 or
  // at least 2^-32, so subnormal results decide nothing).
  static __device__ __forceinline__ bool accept(float u, float t, bool early) {
    const float k = __builtin_rintf(t);
    if (early) {
      const int ki = static_cast<int>(k);
      if (u <= __builtin_ldexpf(1.0f, ki - 1)) return true;
      if (!(u < __builtin_ldexpf(1.0f, ki + 1))) return false;
    }
    return u <= exp2_poly32(t - k, k);
  }
  // The opposite of accept(uniform32(w), t, false), branch-free, in the sign
  // bit: p - float(w) with p = 2^t * 2^32 is negative exactly when
  // float(w) > p (a difference of two floats is zero only when they are
  // equal, and rounding keeps its sign; +inf - float(w) = +inf).
  // k = rint(t) comes from the float adder: t + 1.5 2^23 lies in
  // [2^23, 2^24), where floats are the integers, so the sum rounds t to the
  // nearest integer with ties to even, and k is the sum's representation less
  // that of 1.5 2^23.  Valid for |t| < 2^22, which the library checks at
  // initialisation (beta_max log2(e) max_i 2 sum_d |J| < 2^22).
  static __device__ __forceinline__ uint32_t reject_sign(uint32_t w, float t) {
    const float kf = t + 0x1.8p23f;
    const float k = kf - 0x1.8p23f;
    const int ki = __float_as_int(kf) - 0x4B400000;
    const float p = exp2_poly32_x2p32(t - k, ki);
    return __float_as_uint(p - static_cast<float>(w));
  }
  // Heat bath, FP32 form: a = 2^t, t = -(beta log2 e)|dE| (0 below t = -124),
  // u = float(w) 2^-32; flip iff fma(u, a, u) < (dE > 0 ? a : 1).
  // fw = float(w) of the random word; u = fw 2^-32 exactly
  static __device__ __forceinline__ uint64_t heat_bath_lanes_w(float fw, float bl, float dE) {
    const float t = -(bl * __builtin_fabsf(dE));
    const float kf = t + 0x1.8p23f;  // k = rint(t) from the adder, as in reject_sign
    const float k = kf - 0x1.8p23f;
    const float p = __builtin_ldexpf(exp2_frac32(t - k), __float_as_int(kf) - 0x4B400000);
    const float a = t >= -124.0f ? p : 0.0f;
    const float u = fw * 0x1p-32f;
    return __builtin_amdgcn_ballot_w64(__builtin_fmaf(u, a, u) < (dE > 0.0f ? a : 1.0f));
  }
  static __device__ __forceinline__ float flip_sign(float v, uint32_t s) {
    return __uint_as_float((s & 0x80000000u) ^ __float_as_uint(v));
  }
};

__device__ __forceinline__ double neg_if64(double v, uint32_t bit) {
  const unsigned long long sign = static_cast<unsigned long long>(bit) << 63;
  return __longlong_as_double(static_cast<long long>(static_cast<unsigned long long>(__double_as_longlong(v)) ^ sign));
}

// ---------------------------------------------------------------- lattice helpers
struct Site {
  int i, x, y, z;
};
__device__ __forceinline__ Site site_of(int i, int L) {
  const int x = i % L, yz = i / L;
  return Site{i, x, yz % L, yz / L};
}
// Natural index of the neighbour in direction d (+x,-x,+y,-y,+z,-z).
__device__ __forceinline__ int neighbour(const Site& s, int d, int L) {
  const int L2 = L * L;
  switch (d) {
    case 0: return s.x + 1 < L ? s.i + 1 : s.i - (L - 1);
    case 1: return s.x > 0 ? s.i - 1 : s.i + (L - 1);
    case 2: return s.y + 1 < L ? s.i + L : s.i - L * (L - 1);
    case 3: return s.y > 0 ? s.i - L : s.i + L * (L - 1);
    case 4: return s.z + 1 < L ? s.i + L2 : s.i - L2 * (L - 1);
    default: return s.z > 0 ? s.i - L2 : s.i + L2 * (L - 1);
  }
}
// Word index (within one clone-word plane) of natural site i.
__device__ __forceinline__ int plane_idx(int i, int colour, int Vh) { return colour * Vh + (i >> 1); }
__device__ __forceinline__ int colour_of(const Site& s) { return (s.x + s.y + s.z) & 1; }

__device__ __forceinline__ int word_of(const Geo& g, int clone) {
  return clone < g.NPT ? (clone >> 5) : g.NWPT + ((clone - g.NPT) >> 5);
}
__device__ __forceinline__ int bit_of(const Geo& g, int clone) {
  return clone < g.NPT ? (clone & 31) : ((clone - g.NPT) & 31);
}

// ---------------------------------------------------------------- LDS layout
struct Lds {
  uint32_t* sp;   // [NW][V]
  uint32_t* lab;  // [2*16*NPT] energy partials
  int32_t* cat;   // [NR][NT]
  int32_t* head;  // [NR]
  double* E;      // [NPT + NR] energies: PT clones, then the reservoir FIFO heads
  void* bcl;      // [C] beta per clone (FP)
  uint8_t* rt;    // [NPT]
  int32_t* qacc;  // [NT][npairs] packed Q' | Q_l' << 16
  int32_t* misc;  // [64]
};

__host__ __device__ inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct LdsPlan {
  size_t sp, lab, cat, head, E, bcl, rt, qacc, misc, total;
};
__host__ __device__ inline LdsPlan plan_lds(const Geo& g, int fp_bytes) {
  LdsPlan p{};
  size_t o = 0;
  const int npairs = g.NR * (g.NR - 1) / 2;
  p.sp = o;   o = align_up(o + sizeof(uint32_t) * size_t(g.NW) * g.V, 16);
  const size_t red_words = size_t(2) * kMaxWaves * (g.NPT + g.NR);  // energies of PT clones + reservoir heads
  p.lab = o;  o = align_up(o + sizeof(uint32_t) * red_words, 16);
  p.cat = o;  o = align_up(o + sizeof(int32_t) * size_t(g.NR) * g.NT, 16);
  p.head = o; o = align_up(o + sizeof(int32_t) * size_t(g.NR), 16);
  p.E = o;    o = align_up(o + sizeof(double) * size_t(g.NPT + g.NR), 16);
  p.bcl = o;  o = align_up(o + size_t(fp_bytes) * g.C, 16);
  p.rt = o;   o = align_up(o + size_t(g.NPT), 16);
  p.qacc = o; o = align_up(o + sizeof(int32_t) * 2 * size_t(g.NT) * (npairs > 0 ? npairs : 1), 16);
  p.misc = o; o = align_up(o + sizeof(int32_t) * 64, 16);
  p.total = o;
  return p;
}

extern __shared__ __align__(16) unsigned char lds_raw[];

// Views into the dynamic LDS allocation; every phase rebuilds its own (a few
// integer operations) instead of receiving a struct by reference.
__device__ __forceinline__ Lds lds_view(const Geo& g, int fp_bytes) {
  const LdsPlan plan = plan_lds(g, fp_bytes);
  Lds s;
  s.sp = reinterpret_cast<uint32_t*>(lds_raw + plan.sp);
  s.lab = reinterpret_cast<uint32_t*>(lds_raw + plan.lab);
  s.cat = reinterpret_cast<int32_t*>(lds_raw + plan.cat);
  s.head = reinterpret_cast<int32_t*>(lds_raw + plan.head);
  s.E = reinterpret_cast<double*>(lds_raw + plan.E);
  s.bcl = lds_raw + plan.bcl;
  s.rt = lds_raw + plan.rt;
  s.qacc = reinterpret_cast<int32_t*>(lds_raw + plan.qacc);
  s.misc = reinterpret_cast<int32_t*>(lds_raw + plan.misc);
  return s;
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x / kWave; }

__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) v += __shfl_xor(v, off, kWave);
  return v;
}
__device__ __forceinline__ int wave_incl_scan(int v) {
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int o = __shfl_up(v, off, kWave);
    if (lane_id() >= off) v += o;
  }
  return v;
}

// Exclusive prefix over the workgroup; *total gets the sum.  Uses misc[0..31].
__device__ int block_exclusive_scan(int v, int32_t* misc, int* total) {
  const int incl = wave_incl_scan(v);
  const int nw = (blockDim.x + kWave - 1) / kWave;
  if (lane_id() == kWave - 1) misc[wave_id()] = incl;
  __syncthreads();
  int before = 0, all = 0;
  for (int w = 0; w < nw; ++w) {
    const int m = misc[w];
    if (w < wave_id()) before += m;
    all += m;
  }
  __syncthreads();
  *total = all;
  return before + incl - v;
}

// ---------------------------------------------------------------- union-find
// Lock-free union-find in LDS.  Every entry that is read is a run start
// initialised to itself before the unions start, and every write keeps
// lab[x] <= x with equality only at roots: links go from a root to a smaller
// site of the same cluster (atomicMin), and find() splits paths as it walks
// (lab[x] := lab[lab[x]] <= lab[x] < x).  Chains therefore strictly decrease,
// a find ends within x steps, and the surviving root of a cluster is its
// smallest site.  A racing store can only replace a parent by another
// ancestor-or-relinked site that is smaller and in the same cluster, which
// keeps both properties; a link that loses a race is retried from the value
// atomicMin returned.  Each loop has a single exit condition: the exec-mask
// bookkeeping of divergent loops is scalar work that competes for issue.
__device__ __forceinline__ int find_root(uint32_t* lab, int x) {
  int p = static_cast<int>(lab[x]);
  while (p != x) {
    const int gp = static_cast<int>(lab[p]);
    lab[x] = static_cast<uint32_t>(gp);  // path splitting
    x = p;
    p = gp;
  }
  return x;
}
// The same walk without stores, for the pass that writes every run start's
// final root once the unions are over.  There each entry is written only by
// the work-item that owns it, and only with its root, so a concurrent reader
// sees either the entry's earlier parent or that root: both lead to the same
// root.  A path-splitting find there could store a stale grandparent over an
// owner's root after the owner wrote it.
__device__ __forceinline__ int find_root_readonly(const uint32_t* lab, int x) {
  int p = static_cast<int>(lab[x]);
  while (p != x) {
    x = p;
    p = static_cast<int>(lab[x]);
  }
  return x;
}
// Joins the clusters of a and b.  Every failed link replaces the larger root
// by the smaller value found in its entry, so the larger of the two roots
// strictly decreases and the loop ends within V rounds; the bound only guards
// that argument (reported as an error).
__device__ __forceinline__ void unite(uint32_t* lab, int a, int b, int V, bool* bad) {
  bool linked = false;
  for (int n = 0; !linked && n < V + 2; ++n) {
    a = find_root(lab, a);
    b = find_root(lab, b);
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    const int old = lo == hi ? hi : static_cast<int>(atomicMin(&lab[hi], static_cast<uint32_t>(lo)));
    linked = old == hi;
    a = lo;
    b = old;
  }
  if (!linked) *bad = true;
}

// ---------------------------------------------------------------- the kernel
// Own sites of a work-item: the CH consecutive natural sites starting at
// threadIdx.x * CH (CH/2 of each colour, since L is even).
template <int CH>
struct Own {
  int first;
  bool owns;
  __device__ __forceinline__ Own(int V) : first(static_cast<int>(threadIdx.x) * CH), owns(first < V) {}
  // with several work-items per chunk of sites: chunk index `chunk`
  __device__ __forceinline__ Own(int V, int chunk) : first(chunk * CH), owns(first < V) {}
};

template <typename FP>
__device__ void rebuild_beta(const Geo& g, const Lds& s, const FP* beta) {
  FP* bc = static_cast<FP*>(s.bcl);
  for (int x = threadIdx.x; x < g.NPT; x += blockDim.x) {
    const int r = x / g.NT, k = x % g.NT;
    bc[s.cat[r * g.NT + k]] = beta[k];
  }
  for (int x = threadIdx.x; x < g.NER; x += blockDim.x) bc[g.NPT + x] = beta[g.NT - 1];
}

// ------------------------------------------------------------------ Metropolis
// Couplings of one site as the sweep uses them.  The local field is summed
// axis by axis, h = ((t[+x] + t[-x]) + (t[+y] + t[-y])) + (t[+z] + t[-z]) with
// t[d] = J_d s_i s_j(d) (the s_i factor makes dE = 2h).  With r_d = s_i s_j(d)
// and the couplings A = J[+], B = J[-] of an axis, the axis sum is r_+ (A + B)
// where r_+ = r_-, and r_+ (A - B) where they differ; rounding is symmetric,
// so the signed sum rounded once equals r_+ times the rounded A + B or A - B.
// FP32 stores A + B and A - B per axis; FP64 stores J_d per direction.  Every
// stored value is doubled (exact), so the same sums yield dE = 2h with
// identical rounding.  The signs of the couplings live in these values, so
// the sign words of a word are built from the spin words alone.
template <typename FP>
struct SiteJ {
  FP v[6];  // FP32: 2(A_x + B_x), 2(A_x - B_x), 2(A_y + B_y), ...; FP64: 2 J_d for d = 0..5
};

template <typename FP>
__device__ __forceinline__ SiteJ<FP> make_site_j(const FP (&J)[6]) {
  SiteJ<FP> r;
  if constexpr (sizeof(FP) == 4) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      r.v[2 * a] = 2.0f * (J[2 * a] + J[2 * a + 1]);
      r.v[2 * a + 1] = 2.0f * (J[2 * a] - J[2 * a + 1]);
    }
  } else {
#pragma unroll
    for (int d = 0; d < 6; ++d) r.v[d] = FP(2) * J[d];
  }
  return r;
}

// Sign words of one 32-clone word at one site: bit b concerns clone clone0+b.
// FP64: x[d] is set where r_d = -1 (own spin and neighbour d differ).  FP32:
// per axis, y where r_+ and r_- differ (the two neighbours differ: the own
// spin cancels) and z where r_+ = -1.
struct WordSigns {
  uint32_t x[6], y[3], z[3];
};

// x + x as one v_add_u32: gfx950 issues it at twice the rate of a left shift
// (v_lshlrev_b32), which the compiler would otherwise choose.
__device__ __forceinline__ uint32_t twice(uint32_t x) {
  uint32_t r;
  asm("v_add_u32 %0, %1, %1" : "=v"(r) : "v"(x));
  return r;
}

// The sign words of a word, shifted so that the bit of the clone being
// updated sits at bit 31; one doubling per attempt moves on to the next lower
// clone.  FP32: y[0..2] then z[0..2]; FP64: x[0..5].
struct RunSigns {
  uint32_t s[6];
};
template <typename FP>
__device__ __forceinline__ RunSigns run_signs(const WordSigns& ws, int b_top) {
  RunSigns r;
  const uint32_t sh = 31u - static_cast<uint32_t>(b_top);
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    if constexpr (sizeof(FP) == 4) {
      r.s[a] = (a < 3 ? ws.y[a] : ws.z[a - 3]) << sh;
    } else {
      r.s[a] = ws.x[a] << sh;
    }
  }
  return r;
}

// attempt_group: the Metropolis attempts of the G clones that draw on one
// Philox block (random-number indices n = grp*G + j, j from G-1 down to 0),
// with their clone factors; in a partial last block of a word the surplus
// attempts are discarded by the caller.  Accept iff dE <= 0 or
// u < exp(-beta dE).  kMaybeEarly: clones colder than the early-out threshold
// may decide from the binade of exp(x).  kHB: heat-bath test instead of
// Metropolis (no early-out).  Each decision is shifted in at bit 0 of
// `flips`.  `rs` holds the sign words positioned for the group's first
// (highest) clone and is advanced past the group.
// attempt_group shifts in reject bits instead of accept bits (FP32 Metropolis
// without early-out).
template <typename FP, bool kMaybeEarly, bool kHB>
constexpr bool kRejectBits = sizeof(FP) == 4 && !kMaybeEarly && !kHB;

// The clone factors (beta, or beta log2 e) of the G clones of one Philox
// block.
template <typename FP>
struct Betas {
  FP b[sizeof(FP) == 8 ? 2 : 4];
};
// Those of block grp of a word (clone0, n0 as for update_word), one
// contiguous (scalar) load; in a partial last block the surplus entries belong
// to the next clones or to the table's padding, and their decisions are
// discarded.
template <typename FP>
__device__ __forceinline__ Betas<FP> group_betas(const FP* __restrict__ bc, int clone0, int grp, int n0) {
  constexpr int G = sizeof(FP) == 8 ? 2 : 4;
  const FP* __restrict__ bg = bc + (clone0 + grp * G - n0);
  Betas<FP> r;
#pragma unroll
  for (int j = 0; j < G; ++j) r.b[j] = bg[j];
  return r;
}

// FP64 Metropolis (branch-free form): decisions come from the float bound
// on exp.  With kDefer the lanes it leaves open are added to `open` and the
// caller redoes the word with kExact (the FP64 polynomial for every test) if
// any lane was; without, a group with an open lane takes the polynomial at
// once.  fw: float(w) of the block's words, read by the FP32 Metropolis test
// without early-out and by the FP32 heat-bath test (the other forms read blk).
template <typename FP, bool kMaybeEarly, bool kHB, bool kExact = false, bool kDefer = false>
__device__ __forceinline__ void attempt_group(const Geo& g, const Betas<FP>& betas, RunSigns& rs,
                                              const SiteJ<FP>& sj, const Block& blk, const Floats4& fw,
                                              int early_beta_bits, uint32_t& flips, uint64_t& open) {
  constexpr int G = sizeof(FP) == 8 ? 2 : 4;  // clones per Philox block
  const FP(&beta)[G] = betas.b;
  if constexpr (kRejectBits<FP, kMaybeEarly, kHB>) {
    // FP32 Metropolis, branch-free: the same steps as reject_sign, taken for
    // the group's clones side by side so that every step offers the SIMD G
    // independent instructions; fw holds float(w) of the block's words
    float t[G], f[G], p[G];
    int k[G];
#pragma unroll
    for (int j = G - 1; j >= 0; --j) {
      float ax[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const uint32_t pick = static_cast<uint32_t>(static_cast<int32_t>(rs.s[a]) >> 31);
        ax[a] = Prec<float>::flip_sign(__uint_as_float(bitfield_insert(pick, __float_as_uint(sj.v[2 * a + 1]),
                                                                       __float_as_uint(sj.v[2 * a]))),
                                       rs.s[3 + a]);
      }
#pragma unroll
      for (int a = 0; a < 6; ++a) rs.s[a] = twice(rs.s[a]);
      t[j] = -(static_cast<float>(beta[j]) * ((ax[0] + ax[1]) + ax[2]));
    }
#pragma unroll
    for (int j = G - 1; j >= 0; --j) {
      const float kf = t[j] + 0x1.8p23f;
      f[j] = t[j] - (kf - 0x1.8p23f);
      k[j] = __float_as_int(kf) - 0x4B400000;
    }
#pragma unroll
    for (int j = G - 1; j >= 0; --j) p[j] = kExp2x2p32[6];
#pragma unroll
    for (int n = 5; n >= 0; --n)
#pragma unroll
      for (int j = G - 1; j >= 0; --j) p[j] = __builtin_fmaf(p[j], f[j], kExp2x2p32[n]);
#pragma unroll
    for (int j = G - 1; j >= 0; --j) {
      const float q = __builtin_ldexpf(p[j], k[j]);
      flips = __builtin_amdgcn_alignbit(flips, __float_as_uint(q - fw.u[j]), 31);
    }
    return;
  }
#pragma unroll
  for (int j = G - 1; j >= 0; --j) {
    FP dE;  // the couplings carry the factor 2: the sum is dE = 2h
    if constexpr (sizeof(FP) == 4) {
      float ax[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        // all ones where r_+ and r_- differ: take A - B, else A + B
        const uint32_t pick = static_cast<uint32_t>(static_cast<int32_t>(rs.s[a]) >> 31);
        ax[a] = Prec<float>::flip_sign(__uint_as_float(bitfield_insert(pick, __float_as_uint(sj.v[2 * a + 1]),
                                                                       __float_as_uint(sj.v[2 * a]))),
                                       rs.s[3 + a]);
      }
      dE = (ax[0] + ax[1]) + ax[2];
    } else {
      FP tt[6];
#pragma unroll
      for (int d = 0; d < 6; ++d) tt[d] = Prec<FP>::flip_sign(sj.v[d], rs.s[d]);
      dE = ((tt[0] + tt[1]) + (tt[2] + tt[3])) + (tt[4] + tt[5]);
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) rs.s[a] = twice(rs.s[a]);
    // beta > 0: comparing the float bit patterns as integers orders them
    const bool early = kMaybeEarly && __float_as_int(static_cast<float>(beta[j])) >= early_beta_bits;
    uint64_t acc_lanes;
    if constexpr (kHB) {
      if constexpr (sizeof(FP) == 8) {
        acc_lanes = Prec<double>::heat_bath_lanes(Prec<double>::u(blk, j & 1), beta[j], dE);
      } else {
        acc_lanes = Prec<float>::heat_bath_lanes_w(fw.u[j], beta[j], dE);
      }
    } else if (early) {
      // cold clone (uniform branch): most tests are decided by the binade
      bool acc = dE <= FP(0);
      if (!acc) {
        FP u;
        if constexpr (sizeof(FP) == 8) {
          u = Prec<double>::u(blk, j & 1);
        } else {
          u = uniform32(j == 0 ? blk.w0 : j == 1 ? blk.w1 : j == 2 ? blk.w2 : blk.w3);
        }
        acc = Prec<FP>::accept(u, -(beta[j] * dE), true);
      }
      acc_lanes = __builtin_amdgcn_ballot_w64(acc);
    } else {
      // branch-free: the polynomial is evaluated for every lane (dE <= 0
      // lanes take the test's first clause; their exp value is unused)
      if constexpr (sizeof(FP) == 8) {
        const uint32_t lo = j & 1 ? blk.w2 : blk.w0, hi = j & 1 ? blk.w3 : blk.w1;
        const double x = -(beta[j] * dE);
        const uint64_t nonpos = __builtin_amdgcn_ballot_w64(dE <= 0.0);
        if constexpr (kExact) {
          acc_lanes = nonpos | Prec<double>::exact_lanes(lo, hi, x, __builtin_rint(x * 0x1.71547652b82fep+0));
        } else if constexpr (kDefer) {
          // fw holds the floats of the block's random bits (to_bits53)
          const typename Prec<double>::Bound b = Prec<double>::bound_lanes(fw.u[j & 1], x, g.exp_lo, g.exp_hi);
          acc_lanes = nonpos | b.sure;
          open |= b.open & ~nonpos;
        } else {
          const typename Prec<double>::Bound b =
              Prec<double>::bound_lanes(Prec<double>::bits53(lo, hi), x, g.exp_lo, g.exp_hi);
          acc_lanes = nonpos | (b.open == 0 ? b.sure
                                            : Prec<double>::exact_lanes(lo, hi, x,
                                                                        __builtin_rint(x * 0x1.71547652b82fep+0)));
        }
      } else {
        // beta[j] holds beta log2 e; u <= 2^t already accepts every dE <= 0.
        const uint32_t wj = j == 0 ? blk.w0 : j == 1 ? blk.w1 : j == 2 ? blk.w2 : blk.w3;
        const uint32_t rej = Prec<float>::reject_sign(wj, -(beta[j] * dE));
        if constexpr (kRejectBits<FP, kMaybeEarly, kHB>) {
          // the reject bit (sign of p - float(w)) shifted in with one
          // v_alignbit_b32; the caller inverts the word
          flips = __builtin_amdgcn_alignbit(flips, rej, 31);
          continue;
        } else {
          // next to early-out clones of the same word: accept bits
          acc_lanes = __builtin_amdgcn_ballot_w64(static_cast<int32_t>(rej) >= 0);
        }
      }
    }
    flips = shift_in(flips, acc_lanes);
  }
}

// The word `b` bytes into a word plane.
__device__ __forceinline__ uint32_t* word_at(uint32_t* plane, int b) {
  return reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(plane) + b);
}

// All attempts of one word (clones clone0 .. clone0+nbits-1, random-number
// indices n0 .. n0+nbits-1 with n0 a multiple of 4) at one site (own word and
// neighbour words at byte offsets self_b and nb[d] of the plane).  beta per
// clone comes from uniform (scalar) loads, or with kOneBeta (a word of
// reservoir clones, all at T_max) is bc[clone0] for every clone, read once.
// Blocks are visited from the last to the first, so clone clone0+b ends at
// bit b of the flip mask; the bits of a partial last block's surplus indices
// land above bit nbits-1 and are masked off.
template <typename FP, bool kMaybeEarly, bool kSplit, bool kHB, bool kOneBeta = false>
__device__ __forceinline__ void update_word(const Geo& g, const FP* __restrict__ bc, uint32_t* plane, int self_b,
                                            const int (&nb)[6], const SiteJ<FP>& sj, uint32_t c0w, uint32_t t,
                                            int sample, int clone0, int n0, int nbits, int early_beta_bits,
                                            int f, int F) {
  constexpr int G = sizeof(FP) == 8 ? 2 : 4;
  const FP b_one = kOneBeta ? bc[clone0] : FP(0);
  auto betas = [&](int grp) {
    if constexpr (kOneBeta) {
      Betas<FP> r;
#pragma unroll
      for (int j = 0; j < G; ++j) r.b[j] = b_one;
      return r;
    } else {
      return group_betas(bc, clone0, grp, n0);
    }
  };
  const uint32_t self = *word_at(plane, self_b);
  WordSigns ws;
  if constexpr (sizeof(FP) == 4) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const uint32_t np = *word_at(plane, nb[2 * a]);
      ws.y[a] = np ^ *word_at(plane, nb[2 * a + 1]);
      ws.z[a] = self ^ np;
    }
  } else {
#pragma unroll
    for (int d = 0; d < 6; ++d) ws.x[d] = self ^ *word_at(plane, nb[d]);
  }
  const int g_lo = n0 / G, g_hi = (n0 + nbits - 1) / G;
  // FP64 Metropolis words whose float bounds left a lane open are redone with
  // the FP64 polynomial (the word's spins are written only at the end); the
  // shared-word form, with few groups per wave, takes the polynomial per group
  constexpr bool kRedo = sizeof(FP) == 8 && !kMaybeEarly && !kHB && !kSplit;
  constexpr bool kUsesFloats = kRejectBits<FP, kMaybeEarly, kHB> || (sizeof(FP) == 4 && kHB);
  uint64_t open = 0;
  if constexpr (!kSplit) {
    // software-pipelined: the Philox block of the next group is computed
    // beside the attempts of the current one (independent work for the SIMD)
    auto groups = [&](auto exact_tag) {
      constexpr bool kExact = decltype(exact_tag)::value;
      uint32_t fl = 0;
      int grp = g_hi;
      // groups run from the highest clone down, one clone per doubling
      RunSigns rs = run_signs<FP>(ws, g_hi * G + G - 1 - n0);
      Block blk = philox10(c0w, t, static_cast<uint32_t>(grp), static_cast<uint32_t>(sample), g.key0, g.key1);
      // the block's words are converted as it is taken up (float(w), or the
      // floats of the FP64 tests' random bits in the deferred pass), so that
      // the next block is produced in their registers
      constexpr bool kBits53 = kRedo && !kExact;
      for (; grp > g_lo; --grp) {
        const Floats4 fw = kUsesFloats ? to_floats(blk) : kBits53 ? to_bits53(blk) : Floats4{};
        const Block next =
            philox10(c0w, t, static_cast<uint32_t>(grp - 1), static_cast<uint32_t>(sample), g.key0, g.key1);
        attempt_group<FP, kMaybeEarly, kHB, kExact, kRedo>(g, betas(grp), rs, sj, blk, fw,
                                                           early_beta_bits, fl, open);
        blk = next;
      }
      const Floats4 fw = kUsesFloats ? to_floats(blk) : kBits53 ? to_bits53(blk) : Floats4{};
      attempt_group<FP, kMaybeEarly, kHB, kExact, kRedo>(g, betas(g_lo), rs, sj, blk, fw,
                                                         early_beta_bits, fl, open);
      return fl;
    };
    uint32_t flips = groups(std::false_type{});
    if constexpr (kRedo) {
      if (open != 0) flips = groups(std::true_type{});
    }
    if constexpr (kRejectBits<FP, kMaybeEarly, kHB>) flips = ~flips;
    if (nbits < 32) flips &= (1u << nbits) - 1u;
    *word_at(plane, self_b) = self ^ flips;
  } else {
    // F waves share the word: this one takes groups g_lo + f, g_lo + f + F, ...;
    // each group's decisions land at their own bits, and the flips of the F
    // work-items (disjoint bits) are combined with an atomic XOR
    const int first = g_lo + f;
    if (first > g_hi) return;
    uint32_t flips = 0;
    int grp = first + (g_hi - first) / F * F;
    Block blk = philox10(c0w, t, static_cast<uint32_t>(grp), static_cast<uint32_t>(sample), g.key0, g.key1);
    for (; grp > first; grp -= F) {
      const Floats4 fw = kUsesFloats ? to_floats(blk) : Floats4{};
      const Block next =
          philox10(c0w, t, static_cast<uint32_t>(grp - F), static_cast<uint32_t>(sample), g.key0, g.key1);
      uint32_t part = 0;
      RunSigns rs = run_signs<FP>(ws, grp * G + G - 1 - n0);
      attempt_group<FP, kMaybeEarly, kHB>(g, betas(grp), rs, sj, blk, fw, early_beta_bits,
                                          part, open);
      if constexpr (kRejectBits<FP, kMaybeEarly, kHB>) part = ~part & ((1u << G) - 1u);
      flips |= part << (G * (grp - g_lo));
      blk = next;
    }
    uint32_t part = 0;
    RunSigns rs = run_signs<FP>(ws, first * G + G - 1 - n0);
    const Floats4 fw = kUsesFloats ? to_floats(blk) : Floats4{};
    attempt_group<FP, kMaybeEarly, kHB>(g, betas(first), rs, sj, blk, fw, early_beta_bits,
                                        part, open);
    if constexpr (kRejectBits<FP, kMaybeEarly, kHB>) part = ~part & ((1u << G) - 1u);
    flips |= part << (G * (first - g_lo));
    if (nbits < 32) flips &= (1u << nbits) - 1u;
    if (flips) atomicXor(word_at(plane, self_b), flips);
  }
}

// All attempts of two 16-clone words at two sites a and b of one colour, in
// one 32-clone pass (FP32): the spin words of a fill bits 0..15 of the words
// the pass works on, those of b bits 16..31, so the pass pays once for what a
// word costs besides its attempts (sign words, pipeline fill and drain).  The
// clones of b are visited first, with b's couplings and Philox counter (c0_b),
// then those of a; the next block is produced beside the current group
// throughout, also across the change of site.  Both words hold clones
// clone0 .. clone0+15 with random-number indices n0 .. n0+15 (n0 a multiple
// of 4); decisions and results are those of two update_word calls.
template <typename FP, bool kMaybeEarly, bool kHB>
__device__ __forceinline__ void update_pair16(const Geo& g, const FP* __restrict__ bc, uint32_t* plane, int self_a,
                                              const int (&nb_a)[6], const SiteJ<FP>& sj_a, uint32_t c0_a, int self_b,
                                              const int (&nb_b)[6], const SiteJ<FP>& sj_b, uint32_t c0_b,
                                              uint32_t t, int sample, int clone0, int n0, int early_beta_bits) {
  static_assert(sizeof(FP) == 4, "two 16-clone words per pass: FP32 forms");
  constexpr int G = 4;
  constexpr bool kUsesFloats = kRejectBits<FP, kMaybeEarly, kHB> || kHB;
  // low half of lo in bits 0..15, low half of hi in bits 16..31
  auto merge = [](uint32_t lo, uint32_t hi) { return __builtin_amdgcn_perm(hi, lo, 0x05040100u); };
  const uint32_t wa = *word_at(plane, self_a), wb = *word_at(plane, self_b);
  const uint32_t self = merge(wa, wb);
  RunSigns rs;  // as run_signs: y[0..2] then z[0..2], bit 31 = the first clone visited
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const uint32_t np = merge(*word_at(plane, nb_a[2 * a]), *word_at(plane, nb_b[2 * a]));
    rs.s[a] = np ^ merge(*word_at(plane, nb_a[2 * a + 1]), *word_at(plane, nb_b[2 * a + 1]));
    rs.s[3 + a] = self ^ np;
  }
  const int g_lo = n0 / G;
  // every reservoir clone sits at T_max: one clone factor for the pass
  const FP b = bc[clone0];
  const Betas<FP> betas{{b, b, b, b}};
  uint32_t fl = 0;
  uint64_t open = 0;
  const uint32_t smp = static_cast<uint32_t>(sample);
  Block blk = philox10(c0_b, t, static_cast<uint32_t>(g_lo + 3), smp, g.key0, g.key1);
  for (int grp = g_lo + 3; grp > g_lo; --grp) {
    const Floats4 fw = kUsesFloats ? to_floats(blk) : Floats4{};
    const Block next = philox10(c0_b, t, static_cast<uint32_t>(grp - 1), smp, g.key0, g.key1);
    attempt_group<FP, kMaybeEarly, kHB>(g, betas, rs, sj_b, blk, fw, early_beta_bits, fl, open);
    blk = next;
  }
  {
    const Floats4 fw = kUsesFloats ? to_floats(blk) : Floats4{};
    const Block next = philox10(c0_a, t, static_cast<uint32_t>(g_lo + 3), smp, g.key0, g.key1);
    attempt_group<FP, kMaybeEarly, kHB>(g, betas, rs, sj_b, blk, fw, early_beta_bits, fl, open);
    blk = next;
  }
  for (int grp = g_lo + 3; grp > g_lo; --grp) {
    const Floats4 fw = kUsesFloats ? to_floats(blk) : Floats4{};
    const Block next = philox10(c0_a, t, static_cast<uint32_t>(grp - 1), smp, g.key0, g.key1);
    attempt_group<FP, kMaybeEarly, kHB>(g, betas, rs, sj_a, blk, fw, early_beta_bits, fl, open);
    blk = next;
  }
  {
    const Floats4 fw = kUsesFloats ? to_floats(blk) : Floats4{};
    attempt_group<FP, kMaybeEarly, kHB>(g, betas, rs, sj_a, blk, fw, early_beta_bits, fl, open);
  }
  if constexpr (kRejectBits<FP, kMaybeEarly, kHB>) fl = ~fl;
  *word_at(plane, self_a) = wa ^ (fl & 0xFFFFu);
  *word_at(plane, self_b) = wb ^ (fl >> 16);
}

// n_pt sweeps of the PT clones and n_er sweeps of the ER clones, interleaved
// sweep by sweep (the classes are independent).
template <typename FP, int CH, bool kSplit, bool kHB>
__device__ __forceinline__ void sweep_phase(const Geo& g, const Lds& s, const FP* Js, const FP* __restrict__ bc,
                                            int sample, uint32_t t, int m_pt0, int n_pt, int m_er0, int n_er,
                                            float early_beta, float beta_cold, int F, int part, int P) {
  // kSplit: F waves share each wave-sized block of site chunks, wave f of the
  // F taking every F-th clone group (wave-uniform, so no divergence); with P
  // workgroups per sample (part = this one's index) the groups are dealt
  // over all P F waves of the sample, part + P f taking every (P F)-th.
  const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kWave);
  const int f = kSplit ? part + P * (wv % F) : 0;
  const int FP_ = P * F;
  const Own<CH> own(g.V, kSplit ? (wv / F) * kWave + lane_id() : static_cast<int>(threadIdx.x));
  // Couplings of own sites in the form the field uses (SiteJ).  FP32 (and
  // FP64 with 2 sites per work-item) keeps both colours in registers for all
  // sweeps of the phase; FP64 with 4 sites reloads the current colour's
  // couplings (L2-resident) at every half-sweep to stay within 128 VGPRs.
  constexpr bool kAllInRegs = sizeof(FP) == 4 || CH == 2;
  constexpr int NC = kAllInRegs ? 2 : 1;
  SiteJ<FP> sj[NC][CH / 2];
  int pq[CH / 2];
#pragma unroll
  for (int q = 0; q < CH / 2; ++q) {
    const Site s0 = site_of(own.owns ? own.first + 2 * q : 0, g.L);
    pq[q] = s0.x | (s0.y << 10) | (s0.z << 20);
  }
  auto load_couplings = [&](int slot, int colour) {
#pragma unroll
    for (int q = 0; q < CH / 2; ++q) {
      const int i0 = own.owns ? own.first + 2 * q : 0;
      const int x0 = pq[q] & 1023, y = (pq[q] >> 10) & 1023, z = pq[q] >> 20;
      const int sel = (y + z + colour) & 1;
      const Site sc{i0 + sel, x0 + sel, y, z};
      FP J[6];
#pragma unroll
      for (int d = 0; d < 6; ++d) {
        const int owner = (d & 1) ? neighbour(sc, d, g.L) : sc.i;
        J[d] = own.owns ? Js[size_t(d >> 1) * g.V + owner] : FP(0);
      }
      sj[slot][q] = make_site_j<FP>(J);
    }
  };
  if constexpr (kAllInRegs) {
    load_couplings(0, 0);
    load_couplings(NC - 1, 1);
  }
  const int early_bits = __float_as_int(early_beta);
  const bool er_early = g.NER > 0 && __float_as_int(static_cast<float>(bc[g.NPT])) >= early_bits;
  // PT clones take the early-out form only if the coldest temperature is
  // below the threshold (beta_cold: beta of T_0 in the units bc holds)
  const bool pt_early = __float_as_int(beta_cold) >= early_bits;
  const int n_m = n_pt > n_er ? n_pt : n_er;
  // random-number index of the first reservoir clone: the first multiple of 4
  // at or above N_PT (PT clones use their own ids)
  const int n_er0 = (g.NPT + 3) / 4 * 4;
  // FP32 with two or more sites of a colour per work-item: a last reservoir
  // word of 16 clones is swept two sites per pass (update_pair16)
  constexpr bool kPairs = sizeof(FP) == 4 && CH >= 4 && !kSplit;
  const int er_pair_words = kPairs && g.NER % 32 == 16 ? 1 : 0;
  for (int mm = 0; mm < n_m; ++mm) {
    const bool pt_on = mm < n_pt, er_on = mm < n_er && g.NER > 0;
    const uint32_t c0pt = ctr_word(0, static_cast<uint32_t>(m_pt0 + mm), kMetro);
    const uint32_t c0er = ctr_word(0, static_cast<uint32_t>(m_er0 + mm), kMetro);
    // one checkerboard half-sweep; the colour is a compile-time constant so
    // that the couplings of both colours stay in registers
    auto half_sweep = [&](auto colour_tag) {
      constexpr int colour = decltype(colour_tag)::value;
      constexpr int slot = kAllInRegs ? colour : 0;
      if constexpr (!kAllInRegs) load_couplings(0, colour);
      if (own.owns) {
        // own sites of this colour: natural index, byte offsets of the own
        // and neighbour words within a word plane (one add per address)
        int site_i[CH / 2], self_bq[CH / 2], nbq[CH / 2][6];
#pragma unroll
        for (int q = 0; q < CH / 2; ++q) {
          const int i0 = own.first + 2 * q;  // x even
          const int x0 = pq[q] & 1023, y = (pq[q] >> 10) & 1023, z = pq[q] >> 20;
          const int sel = (y + z + colour) & 1;
          const Site st{i0 + sel, x0 + sel, y, z};
          site_i[q] = st.i;
#pragma unroll
          for (int d = 0; d < 6; ++d) nbq[q][d] = 4 * plane_idx(neighbour(st, d, g.L), colour ^ 1, g.Vh);
          self_bq[q] = 4 * (colour * g.Vh + (i0 >> 1));
        }
#pragma unroll
        for (int q = 0; q < CH / 2; ++q) {
          const int(&nb)[6] = nbq[q];
          const int self_b = self_bq[q];
          // one word of clones: early-out form or not (a uniform choice per word; never for heat bath)
          // kOne: one clone factor for the whole word (update_word's kOneBeta)
          auto word = [&](auto one_tag, bool early, int w, uint32_t c0, int clone0, int n0, int nbits) {
            constexpr bool kOne = decltype(one_tag)::value;
            if (!kHB && early)
              update_word<FP, !kHB, kSplit, kHB, kOne>(g, bc, s.sp + size_t(w) * g.V, self_b, nb, sj[slot][q],
                                                       c0 | static_cast<uint32_t>(site_i[q]), t, sample, clone0, n0,
                                                       nbits, early_bits, f, FP_);
            else
              update_word<FP, false, kSplit, kHB, kOne>(g, bc, s.sp + size_t(w) * g.V, self_b, nb, sj[slot][q],
                                                        c0 | static_cast<uint32_t>(site_i[q]), t, sample, clone0, n0,
                                                        nbits, early_bits, f, FP_);
          };
          if (pt_on)
            for (int w = 0; w < g.NWPT; ++w)
              word(std::false_type{}, pt_early, w, c0pt, 32 * w, 32 * w, min(32, g.NPT - 32 * w));
          if (er_on)
            for (int w = g.NWPT; w < g.NW - er_pair_words; ++w) {
              const int e0 = 32 * (w - g.NWPT);
              // every reservoir clone sits at T_max: one uniform choice of path
              // per word, and one clone factor where a work-item owns its words
              // and there is no two-site pass (with it, such words are rare;
              // shared words measured no faster with it)
              word(std::integral_constant<bool, !kPairs && !kSplit>{}, er_early, w, c0er, g.NPT + e0, n_er0 + e0,
                   min(32, g.NER - e0));
            }
        }
        if constexpr (kPairs) {
          // the last reservoir word, 16 clones per site: two sites per pass
          if (er_on && er_pair_words) {
            const int w = g.NW - 1, e0 = 32 * (w - g.NWPT);
            uint32_t* plane = s.sp + size_t(w) * g.V;
#pragma unroll
            for (int q = 0; q + 1 < CH / 2; q += 2) {
              const uint32_t ca = c0er | static_cast<uint32_t>(site_i[q]);
              const uint32_t cb = c0er | static_cast<uint32_t>(site_i[q + 1]);
              if (!kHB && er_early)
                update_pair16<FP, !kHB, kHB>(g, bc, plane, self_bq[q], nbq[q], sj[slot][q], ca, self_bq[q + 1],
                                             nbq[q + 1], sj[slot][q + 1], cb, t, sample, g.NPT + e0, n_er0 + e0,
                                             early_bits);
              else
                update_pair16<FP, false, kHB>(g, bc, plane, self_bq[q], nbq[q], sj[slot][q], ca, self_bq[q + 1],
                                              nbq[q + 1], sj[slot][q + 1], cb, t, sample, g.NPT + e0, n_er0 + e0,
                                              early_bits);
            }
          }
        }
      }
    };
    half_sweep(std::integral_constant<int, 0>{});
    __syncthreads();
    half_sweep(std::integral_constant<int, 1>{});
    __syncthreads();
  }
}

// ------------------------------------------------------------------ clusters
// Houdayer moves, row-parallel.  A work-item owns one x-row (L <= 32 sites) of
// one move (pair p, temperature k); hou_moves moves are labelled at once, each
// in its own LDS label array.  Along a row the sites of equal overlap
// q_i = s_i^a s_i^b (bit 1: q = -1) form runs, maximal intervals of equal q
// with x = 0 always starting one.  Only run starts are union-find nodes: runs
// are joined across the periodic +x bond of the row and across the +y and +z
// bonds, once per pair of touching runs.  Unions link a root to a smaller site
// (atomicMin), so the surviving root of a cluster is its smallest site, which
// is always a run start: the canonical root.

struct HouLds {
  uint32_t* sp;    // the sample's PT spin words [NWPT][V]: in LDS, or (rows read from
                   // global memory, flips collected) the words in global memory
  int32_t* cat;    // [NR][NT]
  uint32_t* lab;   // [M][Vp] union-find parents (entries of run starts only), padded site indices
  uint32_t* qrow;  // [M][L^2] overlap bits of every row
  uint32_t* eta;   // [M][ceil(Vp/32)] ACU: the root drew eta = -1
  int32_t* misc;   // [kHouMisc] scan scratch, per-move single-cluster data
  uint32_t* size;  // cluster statistics only: [M][Vp] cluster size at its root
  void* flipm;     // moves only: [C][L^2] sites to flip per move of the chunk and
                   // row (uint16 for L <= 16, else uint32)
  int32_t* wlist;  // moves only: [NWPT + 1] offsets, then [2 C] entries
                   // (move in the chunk | bit << 16) of the clones of each PT word
};
// The union-find works on padded site indices: site x + L row is entry
// x + (L + 1) row, so the rows of consecutive work-items start in different
// LDS banks (their run starts are otherwise L words apart, a multiple of the
// bank count for L = 16 or 32).  Padding keeps the order of sites, so the
// smallest padded index of a cluster is that of its smallest site.
__host__ __device__ inline int hou_vp(const Geo& g) { return g.L * g.L * (g.L + 1); }
constexpr int kHouMisc = 32 + 3 * kMaxHouMoves + 7 * kMaxHouMoves;
// misc layout: [0, 32) block scan; 32 + m: single-cluster first count of move m;
// 32 + kMaxHouMoves: total; 33 + kMaxHouMoves + m: chosen root of move m;
// kStatQ + m: overlap sum Q of move m; kStatKey + 6m + 2(round % 3) + sign:
// the round's largest (size, root) key of move m and overlap sign (three
// buffers: a round's buffer is cleared two rounds ahead, after a barrier that
// every reader of its previous use has passed).

constexpr int kStatQ = 32 + 3 * kMaxHouMoves, kStatKey = kStatQ + kMaxHouMoves;

__host__ __device__ inline int hou_moves(const Geo& g) { return (g.NR / 2) * g.K_acu; }
__host__ __device__ inline size_t hou_mask_bytes(const Geo& g) { return g.L <= 16 ? 2 : 4; }
// LDS of the Houdayer kernel with M moves labelled at once; `lds_rows`: the
// PT spin words in LDS; `stats`: the cluster-size arrays; C > 0 (rows from
// global memory): the flip masks of C moves and the word lists.
__host__ __device__ inline size_t hou_lds_bytes(const Geo& g, int M, bool lds_rows, bool stats = false, int C = 0) {
  size_t o = 0;
  if (lds_rows) o = align_up(o + sizeof(uint32_t) * size_t(g.NWPT) * g.V, 16);
  o = align_up(o + sizeof(int32_t) * size_t(g.NR) * g.NT, 16);
  o = align_up(o + sizeof(uint32_t) * size_t(M) * hou_vp(g), 16);
  o = align_up(o + sizeof(uint32_t) * size_t(M) * g.L * g.L, 16);
  o = align_up(o + sizeof(uint32_t) * size_t(M) * ((hou_vp(g) + 31) / 32), 16);
  o = align_up(o + sizeof(int32_t) * kHouMisc, 16);
  if (stats) o = align_up(o + sizeof(uint32_t) * size_t(M) * hou_vp(g), 16);
  if (C > 0) {
    o = align_up(o + hou_mask_bytes(g) * size_t(C) * g.L * g.L, 16);
    o = align_up(o + sizeof(int32_t) * (size_t(g.NWPT) + 1 + 2 * size_t(C)), 16);
  }
  return o;
}
__device__ __forceinline__ HouLds hou_view(const Geo& g, int M, bool lds_rows, bool stats, int C) {
  HouLds s;
  size_t o = 0;
  s.sp = reinterpret_cast<uint32_t*>(lds_raw + o);
  if (lds_rows) o = align_up(o + sizeof(uint32_t) * size_t(g.NWPT) * g.V, 16);
  s.cat = reinterpret_cast<int32_t*>(lds_raw + o);
  o = align_up(o + sizeof(int32_t) * size_t(g.NR) * g.NT, 16);
  s.lab = reinterpret_cast<uint32_t*>(lds_raw + o);
  o = align_up(o + sizeof(uint32_t) * size_t(M) * hou_vp(g), 16);
  s.qrow = reinterpret_cast<uint32_t*>(lds_raw + o);
  o = align_up(o + sizeof(uint32_t) * size_t(M) * g.L * g.L, 16);
  s.eta = reinterpret_cast<uint32_t*>(lds_raw + o);
  o = align_up(o + sizeof(uint32_t) * size_t(M) * ((hou_vp(g) + 31) / 32), 16);
  s.misc = reinterpret_cast<int32_t*>(lds_raw + o);
  o = align_up(o + sizeof(int32_t) * kHouMisc, 16);
  s.size = reinterpret_cast<uint32_t*>(lds_raw + o);  // valid only when laid out with stats
  if (stats) o = align_up(o + sizeof(uint32_t) * size_t(M) * hou_vp(g), 16);
  s.flipm = lds_raw + o;  // valid only when laid out with C > 0
  if (C > 0) o = align_up(o + hou_mask_bytes(g) * size_t(C) * g.L * g.L, 16);
  s.wlist = reinterpret_cast<int32_t*>(lds_raw + o);
  return s;
}
// The flip mask of the chunk's move mv at row `row` (bit x: flip both clones
// at site x).
__device__ __forceinline__ void hou_store_mask(const Geo& g, const HouLds& s, int mv, int row, uint32_t fl) {
  const size_t i = size_t(mv) * g.L * g.L + row;
  if (g.L <= 16) static_cast<uint16_t*>(s.flipm)[i] = static_cast<uint16_t>(fl);
  else static_cast<uint32_t*>(s.flipm)[i] = fl;
}
__device__ __forceinline__ uint32_t hou_load_mask(const Geo& g, const HouLds& s, int mv, int row) {
  const size_t i = size_t(mv) * g.L * g.L + row;
  return g.L <= 16 ? static_cast<uint32_t>(static_cast<const uint16_t*>(s.flipm)[i])
                   : static_cast<const uint32_t*>(s.flipm)[i];
}

// Bit x set where a run of the row mask q starts (x = 0 always).
__device__ __forceinline__ uint32_t run_starts(uint32_t q, uint32_t full) { return ((q ^ (q << 1)) | 1u) & full; }
// Position of the last run start at or below x.
__device__ __forceinline__ int start_at(uint32_t rs, int x) {
  return 31 - __builtin_clz(rs & ((2u << x) - 1u));  // 2u << 31 wraps to 0: all bits
}

// Spin bits of clone c at the sites (x, y, z), x = 0..L-1, of row y + L z
// (bit x set: spin down).
// The row's sites of each colour are L/2 consecutive plane words (x even:
// colour (y+z)&1, x odd: the other), read four at a time when L % 8 == 0 and
// two at a time when L % 4 == 0.
__device__ __forceinline__ uint32_t clone_row(const Geo& g, const uint32_t* sp, int c, int row) {
  const uint32_t* pl = sp + size_t(word_of(g, c)) * g.V;
  const int b = bit_of(g, c);
  const int yz = row % g.L + row / g.L, i0 = row * g.L;
  uint32_t m = 0;
  if (g.L % 8 == 0) {
    const int c0 = yz & 1;
    const uint4* ev = reinterpret_cast<const uint4*>(pl + c0 * g.Vh + i0 / 2);        // x = 0, 2, 4, ...
    const uint4* od = reinterpret_cast<const uint4*>(pl + (c0 ^ 1) * g.Vh + i0 / 2);  // x = 1, 3, 5, ...
    for (int v = 0; v < g.L / 8; ++v) {
      const uint4 e = ev[v], o = od[v];
      const uint32_t part = ((e.x >> b) & 1u) | (((o.x >> b) & 1u) << 1) | (((e.y >> b) & 1u) << 2) |
                            (((o.y >> b) & 1u) << 3) | (((e.z >> b) & 1u) << 4) | (((o.z >> b) & 1u) << 5) |
                            (((e.w >> b) & 1u) << 6) | (((o.w >> b) & 1u) << 7);
      m |= part << (8 * v);
    }
  } else if (g.L % 4 == 0) {
    const int c0 = yz & 1;
    const uint2* ev = reinterpret_cast<const uint2*>(pl + c0 * g.Vh + i0 / 2);        // x = 0, 2, 4, ...
    const uint2* od = reinterpret_cast<const uint2*>(pl + (c0 ^ 1) * g.Vh + i0 / 2);  // x = 1, 3, 5, ...
    for (int v = 0; v < g.L / 4; ++v) {
      const uint2 e = ev[v], o = od[v];
      const uint32_t part = ((e.x >> b) & 1u) | (((o.x >> b) & 1u) << 1) | (((e.y >> b) & 1u) << 2) |
                            (((o.y >> b) & 1u) << 3);
      m |= part << (4 * v);
    }
  } else {
    for (int x = 0; x < g.L; ++x) m |= ((pl[plane_idx(i0 + x, (x + yz) & 1, g.Vh)] >> b) & 1u) << x;
  }
  return m;
}
// Overlap bits of a row: bit x set where q = s^a s^b = -1.
__device__ __forceinline__ uint32_t row_overlap(const Geo& g, const uint32_t* sp, int a, int b, int row) {
  return clone_row(g, sp, a, row) ^ clone_row(g, sp, b, row);
}

// Positions x where a run of a row (mask q, starts rs) must be joined with a
// run of the next row (mask qn, starts rsn): the bond between the rows has
// equal overlap at both ends, one union per maximal interval in which both
// runs stay the same.
__device__ __forceinline__ uint32_t join_points(uint32_t q, uint32_t rs, uint32_t qn, uint32_t rsn, uint32_t full) {
  const uint32_t eq = ~(q ^ qn) & full;
  return eq & (~(eq << 1) | rs | rsn);
}

// All unions of one row: the periodic +x bond (if the row's first and last
// sites have equal overlap and lie in different runs) and the join points
// with the +y row ry and the +z row rz, in one loop (the wave runs as many
// rounds as its busiest work-item, not the sum of three such maxima).
__device__ __forceinline__ void join_row(const Geo& g, uint32_t* lab, uint32_t q, uint32_t rs, int row, uint32_t qy,
                                         int ry, uint32_t qz, int rz, uint32_t full, bool* bad) {
  const int L = g.L, Lp = g.L + 1;
  const uint32_t rsy = run_starts(qy, full), rsz = run_starts(qz, full);
  uint32_t uy = join_points(q, rs, qy, rsy, full), uz = join_points(q, rs, qz, rsz, full);
  const int xl = 31 - __builtin_clz(rs);
  bool ux = xl > 0 && ((q >> (L - 1)) & 1u) == (q & 1u);
  while (ux || (uy | uz)) {
    int a, b;
    if (ux) {
      a = Lp * row;
      b = Lp * row + xl;
      ux = false;
    } else if (uy) {
      const int x = __builtin_ctz(uy);
      uy &= uy - 1u;
      a = start_at(rs, x) + Lp * row;
      b = start_at(rsy, x) + Lp * ry;
    } else {
      const int x = __builtin_ctz(uz);
      uz &= uz - 1u;
      a = start_at(rs, x) + Lp * row;
      b = start_at(rsz, x) + Lp * rz;
    }
    unite(lab, a, b, hou_vp(g), bad);
  }
}

// Sizes of the kStatTop largest clusters of the majority (clusters whose
// overlap sign is that of the whole lattice, q >= 0 counting as +1) and of the
// minority, after the roots are final (lab of every run start = its root);
// ip0: the row's first entry in the padded union-find arrays.
// Sizes accumulate at the roots; then kStatTop rounds each take the largest
// remaining (size, smaller root) key per move and sign with LDS atomicMax.
// out: [2][kStatTop] sizes, descending, 0 where there are fewer clusters.
// Called by every work-item of the workgroup (it synchronizes).
__device__ void cluster_stats(const Geo& g, const HouLds& s, bool active, int m, int M, uint32_t q, uint32_t rs,
                              int ip0, int32_t* out) {
  const int L = g.L, Vp = hou_vp(g);
  uint32_t* size = s.size + size_t(active ? m : 0) * Vp;
  const uint32_t* lab = s.lab + size_t(active ? m : 0) * Vp;
  if (active) {
    for (uint32_t r = rs; r; r &= r - 1u) {
      const int xs = __builtin_ctz(r);
      const uint32_t rest = r & (r - 1u);
      const int xe = rest ? __builtin_ctz(rest) : L;
      atomicAdd(&size[lab[ip0 + xs]], static_cast<uint32_t>(xe - xs));
    }
    atomicAdd(&s.misc[kStatQ + m], L - 2 * __builtin_popcount(q));
  }
  __syncthreads();
  // q bit (1: q_i = -1) of the majority clusters of this move
  const uint32_t maj = active && s.misc[kStatQ + m] < 0 ? 1u : 0u;
  uint32_t taken = 0;  // bit xs: the root at run start xs has been reported
  for (int round = 0; round < kStatTop; ++round) {
    int32_t* key = s.misc + kStatKey + 6 * m + 2 * (round % 3);
    if (active) {
      uint32_t best[2] = {0u, 0u};
      for (uint32_t r = rs; r; r &= r - 1u) {
        const int xs = __builtin_ctz(r);
        const int i = ip0 + xs;
        if (static_cast<int>(lab[i]) != i || ((taken >> xs) & 1u)) continue;
        const uint32_t k = (size[i] << 16) | (0xFFFFu - static_cast<uint32_t>(i));
        const int sign = ((q >> xs) & 1u) == maj ? 0 : 1;
        best[sign] = k > best[sign] ? k : best[sign];
      }
      if (best[0]) atomicMax(reinterpret_cast<uint32_t*>(&key[0]), best[0]);
      if (best[1]) atomicMax(reinterpret_cast<uint32_t*>(&key[1]), best[1]);
    }
    __syncthreads();
    if (active) {
      const uint32_t k0 = static_cast<uint32_t>(key[0]), k1 = static_cast<uint32_t>(key[1]);
      if (ip0 == 0) {
        out[round] = static_cast<int32_t>(k0 >> 16);
        out[kStatTop + round] = static_cast<int32_t>(k1 >> 16);
      }
      for (uint32_t r = rs; r; r &= r - 1u) {
        const int xs = __builtin_ctz(r);
        const uint32_t tag = 0xFFFFu - static_cast<uint32_t>(ip0 + xs);
        if ((k0 && (k0 & 0xFFFFu) == tag) || (k1 && (k1 & 0xFFFFu) == tag)) taken |= 1u << xs;
      }
      // clear the buffer of round + 2 (last read in round - 1, before this barrier)
      int32_t* ahead = s.misc + kStatKey + 6 * m + 2 * ((round + 2) % 3);
      if (ip0 == 0) ahead[0] = ahead[1] = 0;
    }
  }
}

// LDS rows: the order in which a row visits the sites of its flip mask, from
// x = rot up, wrapping around, with rot different for rows 8 apart.  The rows
// of one wave keep their spin words L/2 apart, so rows 8 apart (L = 16) meet
// in the same LDS bank whenever they flip the same x in the same step.
__device__ __forceinline__ int flip_rotation(int row, int L) { return (2 * (row >> 3)) % L; }
__device__ __forceinline__ uint32_t rotate_mask(uint32_t fl, int rot, int L, uint32_t full) {
  return rot ? ((fl >> rot) | (fl << (L - rot))) & full : fl;
}
// LDS rows: flips clones a and b at plane index j; several moves may touch one
// word at the same time, so the update is atomic.
__device__ __forceinline__ void flip_pair_atomic(const Geo& g, uint32_t* sp, int a, int b, int j) {
  const int wa = word_of(g, a), wb = word_of(g, b);
  const uint32_t ma = 1u << bit_of(g, a), mb = 1u << bit_of(g, b);
  if (wa == wb) {
    atomicXor(&sp[size_t(wa) * g.V + j], ma | mb);
  } else {
    atomicXor(&sp[size_t(wa) * g.V + j], ma);
    atomicXor(&sp[size_t(wb) * g.V + j], mb);
  }
}
// The flips of a row's mask fl for move (a, b): on the LDS words at once, or
// collected as the chunk's mask of the move.
template <bool kLdsRows>
__device__ __forceinline__ void hou_flip_row(const Geo& g, const HouLds& s, int a, int b, int row, uint32_t fl,
                                             int chunk_move) {
  if constexpr (kLdsRows) {
    const int L = g.L, y = row % L, z = row / L, i0 = row * L;
    const uint32_t full = L == 32 ? 0xFFFFFFFFu : (1u << L) - 1u;
    const int rot = flip_rotation(row, L);
    for (fl = rotate_mask(fl, rot, L, full); fl; fl &= fl - 1u) {
      const int xr = __builtin_ctz(fl) + rot, x = xr >= L ? xr - L : xr;
      flip_pair_atomic(g, s.sp, a, b, plane_idx(i0 + x, (x + y + z) & 1, g.Vh));
    }
  } else {
    hou_store_mask(g, s, chunk_move, row, fl);
  }
}

// The flips of moves m0 .. m1-1 (the moves of one step use disjoint clones,
// so they commute and can wait until a chunk of them is labelled): for each
// PT word, the list of (move, bit) of its clones, then every work-item XORs
// into the words of its sites the bits whose move flipped that site (global
// memory, one read-modify-write per word and site that changes).  Called by
// every work-item; it synchronizes.
__device__ void hou_apply_flips(const Geo& g, const HouLds& s, uint32_t* gsp, int m0, int m1) {
  const int L = g.L;
  int32_t* off = s.wlist;                // [NWPT + 1]
  int32_t* ent = s.wlist + g.NWPT + 1;   // [2 (m1 - m0)]
  auto clone_of = [&](int m, int side) {
    const int p = m / g.K_acu, k = m - p * g.K_acu;
    return s.cat[(2 * p + side) * g.NT + k];
  };
  for (int w = threadIdx.x; w < g.NWPT; w += blockDim.x) {
    int n = 0;
    for (int m = m0; m < m1; ++m)
      n += (word_of(g, clone_of(m, 0)) == w ? 1 : 0) + (word_of(g, clone_of(m, 1)) == w ? 1 : 0);
    off[w + 1] = n;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    off[0] = 0;
    for (int w = 0; w < g.NWPT; ++w) off[w + 1] += off[w];
  }
  __syncthreads();
  for (int w = threadIdx.x; w < g.NWPT; w += blockDim.x) {
    int n = off[w];
    for (int m = m0; m < m1; ++m)
      for (int side = 0; side < 2; ++side) {
        const int c = clone_of(m, side);
        if (word_of(g, c) == w) ent[n++] = (m - m0) | (bit_of(g, c) << 16);
      }
  }
  __syncthreads();
  // one (word, row) per work-item (L <= 16, see houdayer_plan): each entry's
  // row mask is read once and spread over the row's L sites
  const int L2 = L * L;
  for (int item = threadIdx.x; item < g.NWPT * L2; item += blockDim.x) {
    const int w = item / L2, row = item - w * L2;
    const int e0 = off[w], e1 = off[w + 1];
    uint32_t acc[16];
#pragma unroll
    for (int x = 0; x < 16; ++x) acc[x] = 0u;
    for (int e = e0; e < e1; ++e) {
      const int v = ent[e];
      const uint32_t msk = hou_load_mask(g, s, v & 0xFFFF, row);
      const uint32_t b = static_cast<uint32_t>(v) >> 16;
#pragma unroll
      for (int x = 0; x < 16; ++x) acc[x] |= ((msk >> x) & 1u) << b;
    }
    // site x of the row: colour (x + y + z) & 1, plane word row L/2 + x/2
    uint32_t* plane = gsp + size_t(w) * g.V + size_t(row) * (L / 2);
    const int c0 = (row % L + row / L) & 1;
#pragma unroll
    for (int x = 0; x < 16; ++x)
      if (x < L && acc[x]) plane[size_t(c0 ^ (x & 1)) * g.Vh + (x >> 1)] ^= acc[x];
  }
  __syncthreads();
}

// One Houdayer move for every pair p and every k < K_acu (or, with `labels`,
// the canonical labels of every such pair into labels [S][NR/2][K_acu][V]),
// hou_moves moves per pass.
template <bool kLdsRows>
__device__ bool houdayer_moves(const Geo& g, const HouLds& s, int M, int C, int sample, uint32_t t, int32_t* labels,
                               int32_t* stats) {
  const bool flips = !labels && !stats;
  const bool collect = flips && !kLdsRows;  // flips collected per chunk, then applied to global memory
  const int L = g.L, L2 = L * L, V = g.V, Vp = hou_vp(g);
  const uint32_t full = L == 32 ? 0xFFFFFFFFu : (1u << L) - 1u;
  const int n_moves = (g.NR / 2) * g.K_acu;
  const int eta_words = (Vp + 31) / 32;
  const int m = threadIdx.x / L2, row = threadIdx.x % L2;
  // i0: the row's first site; ip0: its entry in the padded union-find arrays
  const int y = row % L, z = row / L, i0 = row * L, ip0 = row * (L + 1);
  bool bad = false;
  for (int base = 0; base < n_moves; base += M) {
    const int mv = base + m;
    const bool active = m < M && mv < n_moves;
    const int p = active ? mv / g.K_acu : 0, k = active ? mv % g.K_acu : 0;
    const int a = s.cat[(2 * p) * g.NT + k], b = s.cat[(2 * p + 1) * g.NT + k];
    const uint32_t slot = static_cast<uint32_t>(p * g.NT + k);
    uint32_t* lab = s.lab + size_t(active ? m : 0) * Vp;
    uint32_t* eta = s.eta + size_t(active ? m : 0) * eta_words;
    // the first move of the current chunk of collected flips (C a multiple of M)
    const int cb = collect ? base - base % C : 0;
    if (collect && cb == base)
      for (int x = threadIdx.x; x < C * L2; x += blockDim.x) hou_store_mask(g, s, x / L2, x % L2, 0u);
    // overlap bits of the row; run starts become singleton roots
    for (int x = threadIdx.x; x < M * eta_words; x += blockDim.x) s.eta[x] = 0u;
    if (stats) {
      for (int x = threadIdx.x; x < M * Vp; x += blockDim.x) s.size[x] = 0u;
      for (int x = threadIdx.x; x < M; x += blockDim.x) s.misc[kStatQ + x] = 0;
      for (int x = threadIdx.x; x < 6 * M; x += blockDim.x) s.misc[kStatKey + x] = 0;
    }
    uint32_t q = 0, rs = 0;
    if (active) {
      q = row_overlap(g, s.sp, a, b, row);
      s.qrow[m * L2 + row] = q;
      rs = run_starts(q, full);
      for (uint32_t r = rs; r; r &= r - 1u) {
        const int ip = ip0 + __builtin_ctz(r);
        lab[ip] = static_cast<uint32_t>(ip);
      }
    }
    __syncthreads();
    // unions: the periodic +x bond of the row, the +y and the +z rows
    if (active) {
      const int ry = (y + 1 == L ? 0 : y + 1) + L * z, rz = y + L * (z + 1 == L ? 0 : z + 1);
      join_row(g, lab, q, rs, row, s.qrow[m * L2 + ry], ry, s.qrow[m * L2 + rz], rz, full, &bad);
    }
    __syncthreads();
    // roots; under ACU every root draws its eta from the block (ACU, root, slot)
    if (active) {
      uint32_t own_roots = 0;  // run starts that are the roots of their clusters
      for (uint32_t r = rs; r; r &= r - 1u) {
        const int x = __builtin_ctz(r);
        const int root = find_root_readonly(lab, ip0 + x);
        lab[ip0 + x] = static_cast<uint32_t>(root);
        own_roots |= root == ip0 + x ? 1u << x : 0u;
      }
      // the coin of a root is keyed by its site index; eta by its padded entry
      if (flips && g.mode == 0)
        for (; own_roots; own_roots &= own_roots - 1u) {
          const int x = __builtin_ctz(own_roots);
          const Block blk = philox10(ctr_word(i0 + x, 0, kAcu), t, slot, sample, g.key0, g.key1);
          const int ip = ip0 + x;
          if (blk.w0 >> 31) atomicOr(&eta[ip >> 5], 1u << (ip & 31));
        }
    }
    if (stats) {
      __syncthreads();
      cluster_stats(g, s, active, m, M, q, rs, ip0,
                    active ? stats + ((size_t(sample) * (g.NR / 2) + p) * g.K_acu + k) * 2 * kStatTop : nullptr);
    } else if (flips && g.mode != 0) {
      // single cluster: the q = -1 cluster of the target-th q = -1 site in
      // site order, target uniform; per-move counts from one block scan
      int total = 0;
      const int cnt = active ? __builtin_popcount(q) : 0;
      const int before = block_exclusive_scan(cnt, s.misc, &total);  // synchronizes
      if (active && row == 0) s.misc[32 + m] = before;
      if (threadIdx.x == 0) s.misc[32 + kMaxHouMoves] = total;
      __syncthreads();
      if (active) {
        const int first = s.misc[32 + m];
        const int last = (m + 1 < M && base + m + 1 < n_moves) ? s.misc[32 + m + 1] : s.misc[32 + kMaxHouMoves];
        const int n_minus = last - first;
        if (n_minus > 0) {
          const Block blk = philox10(ctr_word(0, 0, kHseed), t, slot, sample, g.key0, g.key1);
          const int target = static_cast<int>((static_cast<uint64_t>(blk.w0) * static_cast<uint32_t>(n_minus)) >> 32);
          int rank = target - (before - first);
          if (rank >= 0 && rank < cnt) {
            uint32_t bits = q;
            for (; rank > 0; --rank) bits &= bits - 1u;
            const int x = __builtin_ctz(bits);
            s.misc[32 + kMaxHouMoves + 1 + m] = static_cast<int32_t>(lab[ip0 + start_at(rs, x)]);
          }
        }
      }
      __syncthreads();
      if (active) {
        const int first = s.misc[32 + m];
        const int last = (m + 1 < M && base + m + 1 < n_moves) ? s.misc[32 + m + 1] : s.misc[32 + kMaxHouMoves];
        if (last > first) {
          const uint32_t root = static_cast<uint32_t>(s.misc[32 + kMaxHouMoves + 1 + m]);
          uint32_t fl = 0;
          for (uint32_t r = rs; r; r &= r - 1u) {
            const int xs = __builtin_ctz(r);
            const uint32_t rest = r & (r - 1u);
            const uint32_t run = (rest ? (rest & (0u - rest)) : (full + 1u)) - (1u << xs);  // bits xs .. xe-1
            fl |= lab[ip0 + xs] == root ? run : 0u;
          }
          hou_flip_row<kLdsRows>(g, s, a, b, row, fl, mv - cb);
        }
      }
    } else {
      __syncthreads();
      if (active) {
        if (labels) {
          int32_t* out = labels + ((size_t(sample) * (g.NR / 2) + p) * g.K_acu + k) * V;
          for (int x = 0; x < L; ++x) {
            const int rp = static_cast<int>(lab[ip0 + start_at(rs, x)]);
            out[i0 + x] = rp - rp / (L + 1);  // the root's site index
          }
        } else {
          // all-cluster update: flip both replicas on clusters whose root drew
          // eta = -1; the row's sites to flip are gathered into one mask first
          uint32_t fl = 0;
          for (uint32_t r = rs; r; r &= r - 1u) {
            const int xs = __builtin_ctz(r);
            const uint32_t root = lab[ip0 + xs];
            const uint32_t rest = r & (r - 1u);
            const uint32_t run = (rest ? (rest & (0u - rest)) : (full + 1u)) - (1u << xs);  // bits xs .. xe-1
            fl |= (eta[root >> 5] >> (root & 31)) & 1u ? run : 0u;
          }
          hou_flip_row<kLdsRows>(g, s, a, b, row, fl, mv - cb);
        }
      }
    }
    __syncthreads();
    // a full chunk (or the last moves): flip the spins
    if (collect && (base + M - cb >= C || base + M >= n_moves)) hou_apply_flips(g, s, s.sp, cb, min(cb + C, n_moves));
  }
  return bad;
}

// ------------------------------------------------------------------ energies
// E(c) = -sum_i a_i, a_i = (J_x[i] s_i s_{i+x} + J_y[i] s_i s_{i+y}) + J_z[i] s_i s_{i+z}
// in double, summed by a pairwise tree in natural site order (own chunk, then
// across the wave's lanes, then across the waves), padded with +0.0 to a
// power of two.  Writes s.E[0..NPT) and, with `heads`, s.E[NPT + r] for the
// oldest reservoir clone of every group r (s.head must be loaded).
//
// The PT clones are taken 16 at a time from their 32-clone words: a
// work-item reads the words of its sites and their +x, +y, +z neighbours
// once per word and walks the clones' bits with one doubling per clone.  The
// 16 lane trees of a batch run transposed: at the level that adds lanes l and
// l ^ o (o = 1, 2, 4, 8) each lane keeps the half of its clones selected by
// bit o of its lane id and adds its partner's value of them, so after four
// levels lane l holds clone (l & 15) summed over its 16 lanes; levels 16 and
// 32 are ordinary exchanges.  Every addition pairs the same two subtrees as
// the tree does, so the sums are bit-identical to it.
template <int CH>
struct EnergySites {
  double jf[CH][3];
  int self[CH], fn[CH][3];
};

// Pairwise tree over the work-item's CH site terms of one clone.
template <int CH>
__device__ __forceinline__ double own_tree(double (&a)[CH]) {
#pragma unroll
  for (int w = CH; w > 1; w >>= 1) {
#pragma unroll
    for (int j = 0; j < w / 2; ++j) a[j] = a[2 * j] + a[2 * j + 1];
  }
  return a[0];
}

template <typename FP, int CH>
__device__ __forceinline__ void energy_phase(const Geo& g, const FP* Js, bool heads = false) {
  const Lds s = lds_view(g, sizeof(FP));
  const Own<CH> own(g.V);
  EnergySites<CH> es;
#pragma unroll
  for (int j = 0; j < CH; ++j) {
    const int i = own.owns ? own.first + j : 0;
    const Site st = site_of(i, g.L);
    const int col = colour_of(st);
    es.self[j] = plane_idx(i, col, g.Vh);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      es.jf[j][d] = own.owns ? static_cast<double>(Js[size_t(d) * g.V + i]) : 0.0;
      es.fn[j][d] = plane_idx(neighbour(st, 2 * d, g.L), col ^ 1, g.Vh);
    }
  }
  double* red = reinterpret_cast<double*>(s.lab);
  const int nwave = (blockDim.x + kWave - 1) / kWave;
  int nwp = 1;
  while (nwp < nwave) nwp <<= 1;
  // entries: the PT clones, then (heads) the oldest reservoir clone of each group
  const int n_e = g.NPT + (heads ? g.NR : 0);
  const int lane = lane_id();
  // clones per batch: 16 (8 with 8 sites per work-item, for registers)
  constexpr int B = CH >= 8 ? 8 : 16;
  for (int c0 = 0; c0 < g.NPT; c0 += B) {
    // bond-sign words of this batch's word: bit b set where the two spins of
    // a bond differ (the term is -J), moved so that clone c0 + B - 1 sits at
    // bit 31; element k of v is clone c0 + B - 1 - k
    const uint32_t* plane = s.sp + size_t(c0 >> 5) * g.V;
    uint32_t xs[CH][3];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const uint32_t si = own.owns ? plane[es.self[j]] : 0u;
#pragma unroll
      for (int d = 0; d < 3; ++d) xs[j][d] = (own.owns ? si ^ plane[es.fn[j][d]] : 0u) << (32 - B - (c0 & 31));
    }
    double v[B];
#pragma unroll
    for (int k = 0; k < B; ++k) {
      double a[CH];
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        const double tx = neg_if64(es.jf[j][0], xs[j][0] >> 31);
        const double ty = neg_if64(es.jf[j][1], xs[j][1] >> 31);
        const double tz = neg_if64(es.jf[j][2], xs[j][2] >> 31);
        a[j] = (tx + ty) + tz;
      }
      v[k] = own_tree<CH>(a);
#pragma unroll
      for (int j = 0; j < CH; ++j)
#pragma unroll
        for (int d = 0; d < 3; ++d) xs[j][d] += xs[j][d];
    }
    // transposed lane tree over lanes B m .. B m + B - 1
#pragma unroll
    for (int o = 1, n = B; o < B; o <<= 1, n >>= 1) {
      const bool upper = (lane & o) != 0;
#pragma unroll
      for (int k = 0; k < n / 2; ++k) {
        // keep element 2k + upper, send the other one
        const double keep = upper ? v[2 * k + 1] : v[2 * k];
        const double send = upper ? v[2 * k] : v[2 * k + 1];
        v[k] = keep + __shfl_xor(send, o, kWave);
      }
    }
    double t = v[0];  // element lane % B, summed over the lane's group of B
#pragma unroll
    for (int o = B; o < kWave; o <<= 1) t = t + __shfl_xor(t, o, kWave);
    const int c = c0 + B - 1 - (lane % B);
    if (lane < B && c < g.NPT) red[wave_id() * n_e + c] = t;
  }
  // the reservoir heads, one clone at a time
  for (int c = g.NPT; c < n_e; ++c) {
    const int clone = g.NPT + (c - g.NPT) * g.NERG + s.head[c - g.NPT];
    const uint32_t* plane = s.sp + size_t(word_of(g, clone)) * g.V;
    const int b = bit_of(g, clone);
    double a[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      a[j] = 0.0;
      if (own.owns) {
        const uint32_t si = plane[es.self[j]] >> b;
        const double tx = neg_if64(es.jf[j][0], (si ^ (plane[es.fn[j][0]] >> b)) & 1u);
        const double ty = neg_if64(es.jf[j][1], (si ^ (plane[es.fn[j][1]] >> b)) & 1u);
        const double tz = neg_if64(es.jf[j][2], (si ^ (plane[es.fn[j][2]] >> b)) & 1u);
        a[j] = (tx + ty) + tz;
      }
    }
    double v = own_tree<CH>(a);
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) v = v + __shfl_xor(v, off, kWave);
    if (lane == 0) red[wave_id() * n_e + c] = v;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < n_e; c += blockDim.x) {
    for (int q = nwave; q < nwp; ++q) red[q * n_e + c] = 0.0;
    for (int width = nwp; width > 1; width >>= 1)
      for (int q = 0; q < width / 2; ++q)
        red[q * n_e + c] = red[(2 * q) * n_e + c] + red[(2 * q + 1) * n_e + c];
    s.E[c] = -red[c];
  }
  __syncthreads();
}

// ------------------------------------------------------------------ PT + ER
template <typename FP, int CH>
__device__ __forceinline__ void pt_phase(const Geo& g, const State& st, int sample, uint32_t t, int do_reservoir,
                                      const FP* beta_fp) {
  const Lds s = lds_view(g, sizeof(FP));
  const bool exchange = do_reservoir && g.NERG > 0;
  energy_phase<FP, CH>(g, static_cast<const FP*>(st.J) + size_t(sample) * 3 * g.V, exchange);
  const Own<CH> own(g.V);
  const int NT = g.NT;
  if (static_cast<int>(threadIdx.x) < g.NR) {
    const int r = threadIdx.x;
    int32_t* at = s.cat + r * NT;
    const size_t base = (size_t(sample) * g.NR + r) * (NT - 1);
    for (int k = 0; k < NT - 1; ++k) {
      const double x = (st.beta64[k] - st.beta64[k + 1]) * (s.E[at[k]] - s.E[at[k + 1]]);
      const Block blk = philox10(ctr_word(k, 0, kPt), t, r, sample, g.key0, g.key1);
      const bool acc = (x >= 0.0) || (uniform53(blk.w0, blk.w1) < exp_neg64(x));
      st.pt_last[base + k] = static_cast<uint8_t>(acc);
      st.pt_count[base + k] += static_cast<uint32_t>(acc);
      if (acc) {
        const int32_t tmp = at[k];
        at[k] = at[k + 1];
        at[k + 1] = tmp;
      }
    }
    // round trips: left T_max -> touched T_min -> back at T_max
    if (s.rt[at[0]] == 1) s.rt[at[0]] = 2;
    if (s.rt[at[NT - 1]] == 2)  // groups finish concurrently: count atomically
      atomicAdd(reinterpret_cast<unsigned long long*>(&st.rt_count[sample]), 1ull);
    s.rt[at[NT - 1]] = 1;
  }
  for (int c = threadIdx.x; c < g.NPT; c += blockDim.x) st.pt_energy[size_t(sample) * g.NPT + c] = s.E[c];
  __syncthreads();
  // energy of every PT clone's configuration after the step: the clone at T_max
  // of group r receives the configuration (and energy) of the reservoir head
  for (int c = threadIdx.x; c < g.NPT; c += blockDim.x) {
    double e = s.E[c];
    if (exchange)
      for (int r = 0; r < g.NR; ++r)
        if (s.cat[r * NT + NT - 1] == c) e = s.E[g.NPT + r];
    st.e_now[size_t(sample) * g.NPT + c] = e;
  }
  if (exchange) {
    // the configuration at T_max and the oldest reservoir configuration trade places
    for (int r = 0; r < g.NR; ++r) {
      const int a = s.cat[r * NT + NT - 1];
      const int b = g.NPT + r * g.NERG + s.head[r];
      if (own.owns) {
        const int wa = word_of(g, a), wb = word_of(g, b), ba = bit_of(g, a), bb = bit_of(g, b);
#pragma unroll
        for (int j = 0; j < CH; ++j) {
          const int i = own.first + j;
          const int jj = plane_idx(i, colour_of(site_of(i, g.L)), g.Vh);
          const uint32_t va = (s.sp[size_t(wa) * g.V + jj] >> ba) & 1u;
          const uint32_t vb = (s.sp[size_t(wb) * g.V + jj] >> bb) & 1u;
          if (va != vb) {
            s.sp[size_t(wa) * g.V + jj] ^= 1u << ba;
            s.sp[size_t(wb) * g.V + jj] ^= 1u << bb;
          }
        }
      }
    }
    __syncthreads();
    if (static_cast<int>(threadIdx.x) < g.NR) s.head[threadIdx.x] = (s.head[threadIdx.x] + 1) % g.NERG;
  }
  __syncthreads();
  rebuild_beta<FP>(g, s, beta_fp);
  __syncthreads();
}

// ------------------------------------------------------------------ observables
// Overlaps of every replica pair at every temperature, row-parallel: KC
// temperatures at a time, one work-item per (temperature, x-row).  The row
// masks of the N_r clones at each temperature go through LDS (cm,
// [KC][NR][L^2]) so that every row meets its +y and +z neighbour rows.  Per
// pair and row, with q the overlap bits (1: q_i = -1), the row adds
// 2(L - |q|) to Q' and 2(3L - |q ^ q(+x)| - |q ^ q(+y)| - |q ^ q(+z)|) to Q_l'
// (|.| = popcount), packed into s.qacc as in the per-site form.
__device__ void overlaps_rows(const Geo& g, const Lds& s, uint32_t* cm, int KC) {
  const int L = g.L, L2 = L * L, NR = g.NR, NT = g.NT, npairs = NR * (NR - 1) / 2;
  const uint32_t full = L == 32 ? 0xFFFFFFFFu : (1u << L) - 1u;
  const int kk = threadIdx.x / L2, row = threadIdx.x % L2;
  const int y = row % L, z = row / L;
  const int ry = (y + 1 == L ? 0 : y + 1) + L * z, rz = y + L * (z + 1 == L ? 0 : z + 1);
  const bool wave_one_k = L2 % kWave == 0;  // every wave's work-items share kk
  for (int k0 = 0; k0 < NT; k0 += KC) {
    const int k = k0 + kk;
    const bool active = kk < KC && k < NT;
    if (active)
      for (int r = 0; r < NR; ++r) cm[(kk * NR + r) * L2 + row] = clone_row(g, s.sp, s.cat[r * NT + k], row);
    __syncthreads();
    if (active) {
      const uint32_t* c0 = cm + size_t(kk) * NR * L2;
      int pair = 0;
      for (int a = 0; a < NR; ++a) {
        const uint32_t ma = c0[a * L2 + row], may = c0[a * L2 + ry], maz = c0[a * L2 + rz];
        for (int b = a + 1; b < NR; ++b, ++pair) {
          const uint32_t q = ma ^ c0[b * L2 + row];
          const uint32_t qy = may ^ c0[b * L2 + ry], qz = maz ^ c0[b * L2 + rz];
          const uint32_t qx = ((q >> 1) | (q << (L - 1))) & full;  // bit x: q at x + 1 (periodic)
          const int nq = __builtin_popcount(q);
          const int nd = __builtin_popcount(q ^ qx) + __builtin_popcount(q ^ qy) + __builtin_popcount(q ^ qz);
          uint32_t packed = static_cast<uint32_t>(2 * (L - nq)) + (static_cast<uint32_t>(2 * (3 * L - nd)) << 16);
          if (wave_one_k) {
            packed = static_cast<uint32_t>(wave_sum_int(static_cast<int>(packed)));
            if (lane_id() == 0) atomicAdd(reinterpret_cast<uint32_t*>(&s.qacc[k * npairs + pair]), packed);
          } else {
            atomicAdd(reinterpret_cast<uint32_t*>(&s.qacc[k * npairs + pair]), packed);
          }
        }
      }
    }
    __syncthreads();
  }
}

template <typename FP, int CH>
__device__ __forceinline__ void measure_phase(const Geo& g, const State& st, const Obs& ob, int sample, int KC,
                                              bool e_current) {
  const Lds s = lds_view(g, sizeof(FP));
  if (e_current) {
    // the PT step left the energies of the current configurations in e_now
    for (int c = threadIdx.x; c < g.NPT; c += blockDim.x) s.E[c] = st.e_now[size_t(sample) * g.NPT + c];
    __syncthreads();
  } else {
    energy_phase<FP, CH>(g, static_cast<const FP*>(st.J) + size_t(sample) * 3 * g.V);
  }
  const Own<CH> own(g.V);
  const int NT = g.NT, NR = g.NR, npairs = NR * (NR - 1) / 2;
  for (int x = threadIdx.x; x < NT * npairs; x += blockDim.x) s.qacc[x] = 0;
  __syncthreads();
  if (KC > 0) {
    overlaps_rows(g, s, reinterpret_cast<uint32_t*>(lds_raw + plan_lds(g, sizeof(FP)).total), KC);
  } else {
    // Per site and temperature, the spins of the N_r clones there (bit r) and of
    // their three forward neighbours.  Each site adds q_i + 1 in {0, 2} to Q' and
    // sum_d (q_i q_j + 1) in {0..6} to Q_l', packed as Q' | Q_l' << 16 (both
    // fields stay below 2^16 for V <= 8192); Q = Q' - V, Q_l = Q_l' - 3V.
    for (int k = 0; k < NT; ++k) {
      uint32_t m[CH], mn[CH][3];
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        m[j] = 0;
        mn[j][0] = mn[j][1] = mn[j][2] = 0;
        if (own.owns) {
          const Site sti = site_of(own.first + j, g.L);
          const int col = colour_of(sti);
          const int ji = plane_idx(sti.i, col, g.Vh);
          int jn[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) jn[d] = plane_idx(neighbour(sti, 2 * d, g.L), col ^ 1, g.Vh);
          for (int r = 0; r < NR; ++r) {
            const int c = s.cat[r * NT + k];
            const uint32_t* plane = s.sp + size_t(word_of(g, c)) * g.V;
            const int b = bit_of(g, c);
            m[j] |= ((plane[ji] >> b) & 1u) << r;
#pragma unroll
            for (int d = 0; d < 3; ++d) mn[j][d] |= ((plane[jn[d]] >> b) & 1u) << r;
          }
        }
      }
      int pair = 0;
      for (int a = 0; a < NR; ++a)
        for (int b = a + 1; b < NR; ++b, ++pair) {
          uint32_t packed = 0;
          if (own.owns) {
#pragma unroll
            for (int j = 0; j < CH; ++j) {
              const uint32_t qi = ((m[j] >> a) ^ (m[j] >> b)) & 1u;  // 1: q_i = -1
              packed += 2u - 2u * qi;
#pragma unroll
              for (int d = 0; d < 3; ++d) {
                const uint32_t qn = ((mn[j][d] >> a) ^ (mn[j][d] >> b)) & 1u;
                packed += (2u - 2u * (qi ^ qn)) << 16;
              }
            }
          }
          packed = static_cast<uint32_t>(wave_sum_int(static_cast<int>(packed)));
          if (lane_id() == 0 && packed != 0) atomicAdd(reinterpret_cast<uint32_t*>(&s.qacc[k * npairs + pair]), packed);
        }
    }
  }
  __syncthreads();
  const double V = static_cast<double>(g.V);
  for (int k = threadIdx.x; k < NT; k += blockDim.x) {
    double esum = 0.0, e2sum = 0.0, q2sum = 0.0, q4sum = 0.0, qlsum = 0.0, ssum = 0.0;
    for (int r = 0; r < NR; ++r) {
      const double er = s.E[s.cat[r * NT + k]] / V;
      esum += er;
      e2sum += er * er;
    }
    int pair = 0;
    for (int a = 0; a < NR; ++a)
      for (int b = a + 1; b < NR; ++b, ++pair) {
        const uint32_t packed = static_cast<uint32_t>(s.qacc[k * npairs + pair]);
        const int Q = static_cast<int>(packed & 0xFFFFu) - g.V;
        const int QL = static_cast<int>(packed >> 16) - 3 * g.V;
        const double q = static_cast<double>(Q) / V;
        const double ql = static_cast<double>(QL) / (3.0 * V);
        const double q2 = q * q;
        q2sum += q2;
        q4sum += q2 * q2;
        qlsum += ql;
        const double ea = s.E[s.cat[a * NT + k]] / V, eb = s.E[s.cat[b * NT + k]] / V;
        ssum += (ea + eb) / 6.0 + (1.0 - ql) * st.beta64[k];
        atomicAdd(reinterpret_cast<unsigned long long*>(&ob.hist[size_t(k) * (g.V + 1) + (Q + g.V) / 2]), 1ull);
      }
    double* o = ob.acc + (size_t(sample) * NT + k) * 6;
    o[0] += esum;
    o[1] += e2sum;
    o[2] += q2sum;
    o[3] += q4sum;
    o[4] += qlsum;
    o[5] += ssum;
  }
  if (threadIdx.x == 0 && sample == 0) atomicAdd(reinterpret_cast<unsigned long long*>(ob.n_meas), 1ull);
  __syncthreads();
}

// ------------------------------------------------------------------ kernels
// Every phase is its own kernel with its own register budget; each loads the
// parts of the sample it needs from HBM into LDS and writes back what it
// changed.  One workgroup per sample; run.sample_begin offsets the grid.

// Load every spin word and the permutation into LDS.
// n_words: the first n_words spin planes of the sample (all NW by default).
__device__ __forceinline__ void load_spins(const Geo& g, uint32_t* sp, int32_t* cat, const State& st, int sample,
                                           int n_words = -1) {
  const size_t stride = size_t(g.NW) * g.V;
  const size_t words = size_t(n_words < 0 ? g.NW : n_words) * g.V;
  if (words % 4 == 0) {
    const uint4* src = reinterpret_cast<const uint4*>(st.spins + size_t(sample) * stride);
    uint4* dst = reinterpret_cast<uint4*>(sp);
    for (size_t x = threadIdx.x; x < words / 4; x += blockDim.x) dst[x] = src[x];
  } else {
    const uint32_t* gsp = st.spins + size_t(sample) * stride;
    for (size_t x = threadIdx.x; x < words; x += blockDim.x) sp[x] = gsp[x];
  }
  for (int x = threadIdx.x; x < g.NR * g.NT; x += blockDim.x) cat[x] = st.clone_at[size_t(sample) * g.NR * g.NT + x];
}
__device__ __forceinline__ void load_spins(const Geo& g, const Lds& s, const State& st, int sample) {
  load_spins(g, s.sp, s.cat, st, sample);
}
__device__ __forceinline__ void store_spins(const Geo& g, const uint32_t* sp, const State& st, int sample,
                                            int n_words = -1) {
  const size_t stride = size_t(g.NW) * g.V;
  const size_t words = size_t(n_words < 0 ? g.NW : n_words) * g.V;
  if (words % 4 == 0) {
    uint4* dst = reinterpret_cast<uint4*>(st.spins + size_t(sample) * stride);
    const uint4* src = reinterpret_cast<const uint4*>(sp);
    for (size_t x = threadIdx.x; x < words / 4; x += blockDim.x) dst[x] = src[x];
  } else {
    uint32_t* osp = st.spins + size_t(sample) * stride;
    for (size_t x = threadIdx.x; x < words; x += blockDim.x) osp[x] = sp[x];
  }
}
__device__ __forceinline__ void store_spins(const Geo& g, const Lds& s, const State& st, int sample) {
  store_spins(g, s.sp, st, sample);
}

// ------------------------------------------------------------------ MicSA
// ln(u) for 0 < u <= 1 (u normal): u = 2^e m with m in [sqrt(1/2), sqrt(2))
// (exact), f = m - 1 (exact), s = f / (2 + f) (correctly rounded division),
// ln m = 2 atanh(s) = s (2 + 2 s^2/3 + 2 s^4/5 + ...) to s^23 by Horner in
// z = s^2 with fused multiply-adds (|s| < 0.172: the first omitted term is
// below 2^-60 of the sum), then e ln2 in two words (e times the head is
// exact).  Coefficients 2/(2n+1) rounded to double.
constexpr double kAtanhCoef[12] = {0x1.0000000000000p+1, 0x1.5555555555555p-1, 0x1.999999999999ap-2,
                                   0x1.2492492492492p-2, 0x1.c71c71c71c71cp-3, 0x1.745d1745d1746p-3,
                                   0x1.3b13b13b13b14p-3, 0x1.1111111111111p-3, 0x1.e1e1e1e1e1e1ep-4,
                                   0x1.af286bca1af28p-4, 0x1.8618618618618p-4, 0x1.642c8590b2164p-4};
__device__ __forceinline__ double log_unit64(double u) {
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(u));
  int e = static_cast<int>((b >> 52) & 0x7FFull) - 1022;
  double m = __longlong_as_double(static_cast<long long>((b & 0x000FFFFFFFFFFFFFull) | 0x3FE0000000000000ull));
  if (m < 0x1.6a09e667f3bcdp-1) {  // below sqrt(1/2): take m in [sqrt(1/2), 1)
    m *= 2.0;
    e -= 1;
  }
  const double f = m - 1.0;
  const double s = f / (2.0 + f);
  const double z = s * s;
  double p = kAtanhCoef[11];
#pragma unroll
  for (int n = 10; n >= 0; --n) p = __builtin_fma(p, z, kAtanhCoef[n]);
  const double lm = s * p;
  const double de = static_cast<double>(e);
  return __builtin_fma(de, 0x1.62e42feep-1, __builtin_fma(de, 0x1.a39ef35793c76p-33, lm));
}

// MicSA sweeps of the PT clones (App. A.1): each clone carries a walker
// holding an energy W >= 0; a spin flips iff W >= dE, and the walker then
// gives up dE.  The walker is redrawn from its Boltzmann law at the clone's
// temperature, W = T_k (-ln u), at every sweep m with m % micsa_refresh == 0,
// u = (b + 1) 2^-53 from 53 bits b of the block (WALKER, site 0, m, t, clone,
// sample).  The walker makes one clone's sweep sequential, so a lane owns a
// clone and walks its sites in the sweep order (colour 0 in increasing site
// index, then colour 1); the lanes of one 32-clone word take the same site
// at the same time and their flips enter the word through one ballot.  A
// wave's 64 clones fill whole words that no other wave touches, so the
// waves run without barriers.  Sites of one colour are not neighbours, so
// within a half-sweep dE of a site does not depend on the decisions before
// it: the dE of up to 8 sites of a row are formed side by side (independent
// loads and adds), and only the walker's compare-and-subtract runs in
// sequence.  dE is summed as the Metropolis sweep sums it: terms J_d s_i s_j
// in the order ((+x, -x) + (+y, -y)) + (+z, -z), doubled.  kJLds: the
// sample's couplings are staged in LDS (when they fit beside the spins).
constexpr int kMicsaBatch = 8;
template <typename FP, bool kJLds>
__global__ __launch_bounds__(kMaxThreads) void micsa_kernel(Geo g, State st, Run run) {
  const int sample = run.sample_begin + blockIdx.x;
  if (sample >= g.S) return;
  uint32_t* sp = reinterpret_cast<uint32_t*>(lds_raw);  // [NWPT][V]
  size_t o = align_up(sizeof(uint32_t) * size_t(g.NWPT) * g.V, 16);
  int32_t* cat = reinterpret_cast<int32_t*>(lds_raw + o);  // [NR][NT]
  int32_t* kof = cat + g.NR * g.NT;                         // [NPT] temperature index of every clone
  o = align_up(o + sizeof(int32_t) * size_t(g.NR * g.NT + g.NPT), 16);
  const FP* Jg = static_cast<const FP*>(st.J) + size_t(sample) * 3 * g.V;
  FP* Jl = reinterpret_cast<FP*>(lds_raw + o);  // [3][V] when kJLds
  load_spins(g, sp, cat, st, sample, g.NWPT);
  if constexpr (kJLds)
    for (int x = threadIdx.x; x < 3 * g.V; x += blockDim.x) Jl[x] = Jg[x];
  __syncthreads();
  for (int x = threadIdx.x; x < g.NPT; x += blockDim.x) kof[cat[x]] = x % g.NT;
  __syncthreads();
  const FP* Js = kJLds ? Jl : Jg;
  const uint32_t t = *st.t_dev;
  const int L = g.L, L2 = L * L, V = g.V, half = L / 2;
  const int lane = lane_id();
  // blockDim.x is a multiple of 64, so all lanes of a wave take the same trips
  for (int base = 0; base < g.NPT; base += blockDim.x) {
    const int c = base + static_cast<int>(threadIdx.x);
    const bool active = c < g.NPT;
    const int cw = active ? c : base;  // clone whose word and factors inactive lanes read
    const uint32_t* plane = sp + size_t(cw >> 5) * V;
    const int bit = cw & 31;
    const int w_lo = (base + wave_id() * kWave) >> 5;  // words of lanes 0..31 and 32..63
    const double Tk = st.T64[kof[cw]];
    double* wslot = st.walker + size_t(sample) * g.NPT + cw;
    FP W = static_cast<FP>(*wslot);
    for (int mm = 0; mm < run.n_pt; ++mm) {
      const int m = run.m_pt0 + mm;
      if (m % g.micsa_refresh == 0) {
        const Block blk = philox10(ctr_word(0, static_cast<uint32_t>(m), kWalker), t, static_cast<uint32_t>(cw),
                                   static_cast<uint32_t>(sample), g.key0, g.key1);
        const uint64_t b53 = ((static_cast<uint64_t>(blk.w1) << 32) | blk.w0) >> 11;
        W = static_cast<FP>(Tk * -log_unit64(static_cast<double>(b53 + 1) * 0x1p-53));
      }
      for (int colour = 0; colour < 2; ++colour) {
        for (int row = 0; row < L2; ++row) {
          const int y = row % L, z = row / L;
          const int x0 = (y + z + colour) & 1;
          for (int s0 = 0; s0 < half; s0 += kMicsaBatch) {
            FP dE[kMicsaBatch];
#pragma unroll
            for (int k = 0; k < kMicsaBatch; ++k) {
              const int x = x0 + 2 * (s0 + k);
              dE[k] = FP(0);
              if (s0 + k < half) {
                const Site si{row * L + x, x, y, z};
                const uint32_t own = (plane[colour * g.Vh + (si.i >> 1)] >> bit) & 1u;
                FP term[6];
#pragma unroll
                for (int d = 0; d < 6; ++d) {
                  const int n = neighbour(si, d, L);
                  const FP Jd = Js[size_t(d >> 1) * V + ((d & 1) ? n : si.i)];
                  const uint32_t nbit = (plane[(colour ^ 1) * g.Vh + (n >> 1)] >> bit) & 1u;
                  term[d] = (own ^ nbit) ? -Jd : Jd;  // J_d s_i s_j
                }
                dE[k] = FP(2) * (((term[0] + term[1]) + (term[2] + term[3])) + (term[4] + term[5]));
              }
            }
            // the walker, site after site
            uint32_t acc = 0;
#pragma unroll
            for (int k = 0; k < kMicsaBatch; ++k) {
              const bool a = s0 + k < half && active && W >= dE[k];
              if (a) W = W - dE[k];
              acc |= static_cast<uint32_t>(a) << k;
            }
#pragma unroll
            for (int k = 0; k < kMicsaBatch; ++k) {
              if (s0 + k >= half) break;
              const uint64_t flips = __builtin_amdgcn_ballot_w64((acc >> k) & 1u);
              const uint32_t lo = static_cast<uint32_t>(flips), hi = static_cast<uint32_t>(flips >> 32);
              const int j = colour * g.Vh + ((row * L + x0 + 2 * (s0 + k)) >> 1);
              if (lane == 0 && lo) sp[size_t(w_lo) * V + j] ^= lo;
              if (lane == 32 && hi) sp[size_t(w_lo + 1) * V + j] ^= hi;
            }
          }
        }
      }
    }
    if (active) *wslot = static_cast<double>(W);
  }
  __syncthreads();
  store_spins(g, sp, st, sample, g.NWPT);
}

// Row-wise MicSA for L = 2H, 2 <= H <= 8, couplings in LDS.  The same
// sweep, walker and sums as micsa_kernel, reorganised around the lattice
// rows (fixed y, z) of one colour: the couplings are staged in checkerboard
// order (J_d of site i at d V + colour(i) V/2 + i/2, as the spin words), so
// that a row's own words, the other colour's words of the same row and of
// the rows at y -+ 1 and z -+ 1, and the six coupling rows it needs are
// twelve contiguous vectors of H values, read with the widest LDS loads their
// alignment allows (16 bytes when a row holds a multiple of 4 words, else 8
// or 4).
// Within a row x = x0 + 2k; its +x neighbour is the other colour's word
// k + x0 and its -x neighbour (and coupling) word k + x0 - 1, both modulo H.
// Each coupling takes the sign of the neighbour spin (bit 31 of the word
// shifted left by 31 - bit is 1 for a down spin) and the sum of the six takes
// the sign of the updated spin: negation is exact and (-a) + (-b) = -(a + b)
// under round-to-nearest, so dE equals micsa_kernel's sum of the products
// J s_i s_j in the same order bit for bit (a zero dE can differ in its sign,
// which neither W >= dE nor W - dE can tell).  The flips of a site enter the
// row's own words in registers; each row is written back once.
constexpr int kMicsaRowThreads = 256;

template <int N>
__device__ __forceinline__ void lds_words(const uint32_t* p, uint32_t (&v)[N]) {
  if constexpr (N % 4 == 0) {
#pragma unroll
    for (int j = 0; j < N / 4; ++j) {
      const uint4 q = reinterpret_cast<const uint4*>(p)[j];
      v[4 * j] = q.x, v[4 * j + 1] = q.y, v[4 * j + 2] = q.z, v[4 * j + 3] = q.w;
    }
  } else if constexpr (N % 2 == 0) {
#pragma unroll
    for (int j = 0; j < N / 2; ++j) {
      const uint2 q = reinterpret_cast<const uint2*>(p)[j];
      v[2 * j] = q.x, v[2 * j + 1] = q.y;
    }
  } else {
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = p[j];
  }
}
template <int N>
__device__ __forceinline__ void lds_store_words(uint32_t* p, const uint32_t (&v)[N]) {
  if constexpr (N % 4 == 0) {
#pragma unroll
    for (int j = 0; j < N / 4; ++j) reinterpret_cast<uint4*>(p)[j] = make_uint4(v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
  } else if constexpr (N % 2 == 0) {
#pragma unroll
    for (int j = 0; j < N / 2; ++j) reinterpret_cast<uint2*>(p)[j] = make_uint2(v[2 * j], v[2 * j + 1]);
  } else {
#pragma unroll
    for (int j = 0; j < N; ++j) p[j] = v[j];
  }
}
template <int H>
__device__ __forceinline__ void lds_row(const float* p, float (&v)[H]) {
  uint32_t w[H];
  lds_words<H>(reinterpret_cast<const uint32_t*>(p), w);
#pragma unroll
  for (int k = 0; k < H; ++k) v[k] = __uint_as_float(w[k]);
}
template <int H>
__device__ __forceinline__ void lds_row(const double* p, double (&v)[H]) {
  uint32_t w[2 * H];
  lds_words<2 * H>(reinterpret_cast<const uint32_t*>(p), w);
#pragma unroll
  for (int k = 0; k < H; ++k)
    v[k] = __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(w[2 * k + 1]) << 32) | w[2 * k]));
}
// J with its sign flipped where bit 31 of s is set (s has no other bit set).
__device__ __forceinline__ float flip31(float J, uint32_t s) { return __uint_as_float(__float_as_uint(J) ^ s); }
__device__ __forceinline__ double flip31(double J, uint32_t s) {
  return __longlong_as_double(
      static_cast<long long>(static_cast<unsigned long long>(__double_as_longlong(J)) ^ (static_cast<unsigned long long>(s) << 32)));
}

// Words shifted left by sh (the clone's bit to bit 31), two at a time: bit
// 31 of either half of a 64-bit shift comes from that half.
template <int H>
__device__ __forceinline__ void to_bit31(const uint32_t (&v)[H], uint32_t (&out)[H], int sh) {
#pragma unroll
  for (int j = 0; j + 1 < H; j += 2) {
    const uint64_t p = ((static_cast<uint64_t>(v[j + 1]) << 32) | v[j]) << sh;
    out[j] = static_cast<uint32_t>(p);
    out[j + 1] = static_cast<uint32_t>(p >> 32);
  }
  if constexpr (H % 2) out[H - 1] = v[H - 1] << sh;
}

// The six spin-word row vectors of one row of one colour, and the six
// coupling row vectors.
template <int H>
struct MicsaRow {
  uint32_t own[H], xo[H], yp[H], ym[H], zp[H], zm[H];
};
template <typename FP, int H>
struct MicsaJ {
  FP xp[H], xm[H], yp[H], ym[H], zp[H], zm[H];
};

__device__ __forceinline__ int wrap_up(int v, int L) { return v + 1 < L ? v + 1 : 0; }
__device__ __forceinline__ int wrap_down(int v, int L) { return v > 0 ? v - 1 : L - 1; }

// Word offsets (within a plane) of a row of one colour and of the other
// colour's rows it reads: own and xo are the row itself, yp/ym/zp/zm its
// neighbour rows.
struct RowOff {
  int own, xo, yp, ym, zp, zm;
};
// Row y of plane z, colour c; zb, zpb, zmb: the word offsets of planes z,
// z + 1, z - 1 (periodic).
template <int H>
__device__ __forceinline__ RowOff row_off(int y, int zb, int zpb, int zmb, int c) {
  constexpr int L = 2 * H, Vh = L * L * L / 2;
  const int oc = (c ^ 1) * Vh, cc = c * Vh, yh = y * H;
  RowOff o;
  o.own = cc + zb + yh;
  o.xo = oc + zb + yh;
  o.yp = oc + zb + (y + 1 < L ? yh + H : 0);
  o.ym = oc + zb + (y > 0 ? yh - H : (L - 1) * H);
  o.zp = oc + zpb + yh;
  o.zm = oc + zmb + yh;
  return o;
}
// Spin words of a row from the clone word's plane P.
template <int H>
__device__ __forceinline__ void micsa_load(MicsaRow<H>& r, const uint32_t* P, const RowOff& o) {
  lds_words<H>(P + o.own, r.own);
  lds_words<H>(P + o.xo, r.xo);
  lds_words<H>(P + o.yp, r.yp);
  lds_words<H>(P + o.ym, r.ym);
  lds_words<H>(P + o.zp, r.zp);
  lds_words<H>(P + o.zm, r.zm);
}
// Couplings of a row from Jc (checkerboard order): J_x of the row's sites
// and of the other colour's sites of the row (the -x bonds), J_y of the row
// and of the row at y - 1, J_z of the row and of the row at z - 1.
// FP32 couplings read through the scalar data cache (wave-uniform
// addresses; the kernel never writes them).
using ScalarF32 = const __attribute__((address_space(4))) float;
template <int H>
__device__ __forceinline__ void j_row(const float* p, float (&v)[H]) { lds_row<H>(p, v); }
template <int H>
__device__ __forceinline__ void j_row(const double* p, double (&v)[H]) { lds_row<H>(p, v); }
template <int H>
__device__ __forceinline__ void j_row(ScalarF32* p, float (&v)[H]) {
#pragma unroll
  for (int k = 0; k < H; ++k) v[k] = p[k];
}
template <typename FP, int H, typename JP>
__device__ __forceinline__ void micsa_load_j(MicsaJ<FP, H>& j, JP Jc, const RowOff& o) {
  constexpr int L = 2 * H, V = L * L * L;
  j_row<H>(Jc + o.own, j.xp);
  j_row<H>(Jc + o.xo, j.xm);
  j_row<H>(Jc + V + o.own, j.yp);
  j_row<H>(Jc + V + o.ym, j.ym);
  j_row<H>(Jc + 2 * V + o.own, j.zp);
  j_row<H>(Jc + 2 * V + o.zm, j.zm);
}

// dE / 2 of the row's sites with the sign of the updated spin, U[k] for
// x = X0 + 2k: each coupling takes the sign of its neighbour spin, the sum
// that of the updated spin.
template <typename FP, int H, int X0>
__device__ __forceinline__ void micsa_fields(const MicsaRow<H>& r, const MicsaJ<FP, H>& J, int sh, FP (&U)[H]) {
  constexpr uint32_t kSign = 0x80000000u;
  uint32_t xs[H];
  to_bit31<H>(r.xo, xs, sh);
  // two sites at a time, so that only their shifted words are live
#pragma unroll
  for (int j = 0; j < H; j += 2) {
    uint32_t os[2], yps[2], yms[2], zps[2], zms[2];
    const auto pair = [&](const uint32_t(&v)[H], uint32_t(&out)[2]) {
      if (j + 1 < H) {
        const uint64_t q = ((static_cast<uint64_t>(v[j + 1]) << 32) | v[j]) << sh;
        out[0] = static_cast<uint32_t>(q);
        out[1] = static_cast<uint32_t>(q >> 32);
      } else {
        out[0] = v[j] << sh;
        out[1] = 0;
      }
    };
    pair(r.own, os);
    pair(r.yp, yps);
    pair(r.ym, yms);
    pair(r.zp, zps);
    pair(r.zm, zms);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int k = j + i;
      if (k >= H) break;
      const int kp = (k + X0) % H, km = (k + X0 + H - 1) % H;
      const FP u0 = flip31(J.xp[k], xs[kp] & kSign);
      const FP u1 = flip31(J.xm[km], xs[km] & kSign);
      const FP u2 = flip31(J.yp[k], yps[i] & kSign);
      const FP u3 = flip31(J.ym[k], yms[i] & kSign);
      const FP u4 = flip31(J.zp[k], zps[i] & kSign);
      const FP u5 = flip31(J.zm[k], zms[i] & kSign);
      U[k] = flip31(((u0 + u1) + (u2 + u3)) + (u4 + u5), os[i] & kSign);
    }
  }
}

// The walker over one row, site after site; the flips enter own.  W is -inf
// on lanes without a clone, so that they never accept.  W - dE =
// fma(-2, U, W) with dE = 2U exact, rounded once as the difference is; with
// FP32 denormals kept, the rounded difference is >= 0 exactly when W >= dE.
template <typename FP, int H>
__device__ __forceinline__ void micsa_walk(uint32_t (&own)[H], const FP (&U)[H], int hi_shift, FP& W) {
#pragma unroll
  for (int k = 0; k < H; ++k) {
    const FP rest = fma(FP(-2), U[k], W);
    const bool a = rest >= FP(0);
    W = a ? rest : W;
    own[k] ^= static_cast<uint32_t>(__builtin_amdgcn_ballot_w64(a) >> hi_shift);
  }
}

// One row of colour C, whose sites sit at x = X0 + 2k and whose own words
// start at word `own` of the plane, from cur and J; meanwhile the spin words
// of the row at `next` load into nxt and, once this row's sums are formed,
// its couplings into J.  Couplings read through the scalar cache are instead
// loaded for the row itself (at `at`) as it starts: held from one row to the
// next they made the compiler move scalar registers into vector lanes and
// back.  A row never reads a row of its own colour other
// than its own, and the first row of either colour reads none of the rows
// the last row of the other colour writes, so the early loads see final
// words.
template <typename FP, int H, int C, int X0, typename JP>
__device__ __forceinline__ void micsa_step(MicsaRow<H>& cur, MicsaRow<H>& nxt, MicsaJ<FP, H>& J, const uint32_t* P,
                                           uint32_t* Pw, JP Jc, int own, const RowOff& at, const RowOff& next,
                                           int sh, int hi_shift, bool write, FP& W) {
  micsa_load<H>(nxt, P, next);
  FP U[H];
  if constexpr (std::is_same_v<JP, ScalarF32*>) {
    MicsaJ<FP, H> Jr;
    micsa_load_j<FP, H>(Jr, Jc, at);
    micsa_fields<FP, H, X0>(cur, Jr, sh, U);
  } else {
    micsa_fields<FP, H, X0>(cur, J, sh, U);
    micsa_load_j<FP, H>(J, Jc, next);
  }
  micsa_walk<FP, H>(cur.own, U, hi_shift, W);
  if (write) lds_store_words<H>(Pw + own, cur.own);
}

// The rows of plane z of colour C, two per trip so that the buffers
// alternate without copies (L is even); rows with even y have their sites at
// x = XE + 2k, rows with odd y at x = 1 - XE + 2k.  The last row loads the
// first row of the next plane, or of the other colour after the last plane.
template <typename FP, int H, int C, int XE, typename JP>
__device__ __forceinline__ void micsa_plane(MicsaRow<H>& ra, MicsaRow<H>& rb, MicsaJ<FP, H>& J, const uint32_t* P,
                                            uint32_t* Pw, JP Jc, int z, int sh, int hi_shift, bool write,
                                            FP& W) {
  constexpr int L = 2 * H, LH = L * H, Vh = L * L * L / 2;
  const int zb = z * LH, zpb = wrap_up(z, L) * LH, zmb = wrap_down(z, L) * LH;
  // the row after this plane's last: the next plane's first, or the other
  // colour's first after the last plane
  const bool end = z + 1 == L;
  const int nz = end ? 0 : z + 1, nc = end ? C ^ 1 : C;
  const RowOff after = row_off<H>(0, nz * LH, wrap_up(nz, L) * LH, wrap_down(nz, L) * LH, nc);
  for (int y = 0; y < L; y += 2) {
    micsa_step<FP, H, C, XE>(ra, rb, J, P, Pw, Jc, C * Vh + zb + y * H, row_off<H>(y, zb, zpb, zmb, C),
                             row_off<H>(y + 1, zb, zpb, zmb, C), sh, hi_shift, write, W);
    micsa_step<FP, H, C, XE ^ 1>(rb, ra, J, P, Pw, Jc, C * Vh + zb + (y + 1) * H, row_off<H>(y + 1, zb, zpb, zmb, C),
                                 y + 2 < L ? row_off<H>(y + 2, zb, zpb, zmb, C) : after, sh, hi_shift, write, W);
  }
}

// One colour's half-sweep, rows in increasing site order; on entry ra and J
// hold its first row, on exit the first row of the other colour.
template <typename FP, int H, int C, typename JP>
__device__ __forceinline__ void micsa_half_sweep(MicsaRow<H>& ra, MicsaRow<H>& rb, MicsaJ<FP, H>& J,
                                                 const uint32_t* P, uint32_t* Pw, JP Jc, int sh, int hi_shift,
                                                 bool write, FP& W) {
  constexpr int L = 2 * H;
  for (int z = 0; z < L; ++z) {
    if ((z + C) & 1)
      micsa_plane<FP, H, C, 1>(ra, rb, J, P, Pw, Jc, z, sh, hi_shift, write, W);
    else
      micsa_plane<FP, H, C, 0>(ra, rb, J, P, Pw, Jc, z, sh, hi_shift, write, W);
  }
}

// kScalarJ (FP32): the couplings are read in plane order from st.J_plane
// through the scalar data cache and LDS holds only the spin words (at L=16
// with 144 PT clones, 80 KiB: two samples per CU); otherwise LDS also holds
// the permutation and the couplings, rearranged into plane order here.
template <typename FP, int H, bool kScalarJ>
__global__ __launch_bounds__(kMicsaRowThreads) void micsa_row_kernel(Geo g, State st, Run run) {
  static_assert(H >= 2, "the prefetch needs distinct boundary rows");
  static_assert(!kScalarJ || sizeof(FP) == 4, "scalar couplings: FP32 form");
  constexpr int L = 2 * H, V = L * L * L, Vh = V / 2;
  const int sample = run.sample_begin + blockIdx.x;
  if (sample >= g.S) return;
  uint32_t* sp = reinterpret_cast<uint32_t*>(lds_raw);  // [NWPT][V]
  size_t o = align_up(sizeof(uint32_t) * size_t(g.NWPT) * V, 16);
  const int32_t* cat_g = st.clone_at + size_t(sample) * g.NR * g.NT;
  int32_t* cat = reinterpret_cast<int32_t*>(lds_raw + o);  // [NR][NT] (not with kScalarJ)
  int32_t* kof = cat + g.NR * g.NT;                         // [NPT] temperature index of every clone
  o = align_up(o + sizeof(int32_t) * size_t(g.NR * g.NT + g.NPT), 16);
  auto Jc = [&] {
    if constexpr (kScalarJ) {
      return (ScalarF32*)(st.J_plane + size_t(sample) * 3 * V);  // [3][V], plane order (address-space cast)
    } else {
      return reinterpret_cast<FP*>(lds_raw + o);  // [3][V], plane order
    }
  }();
  if constexpr (kScalarJ) {
    const size_t words = size_t(g.NWPT) * V;
    const uint32_t* gsp = st.spins + size_t(sample) * g.NW * V;
    for (size_t x = threadIdx.x; x < words; x += blockDim.x) sp[x] = gsp[x];
  } else {
    load_spins(g, sp, cat, st, sample, g.NWPT);
    const FP* Jg = static_cast<const FP*>(st.J) + size_t(sample) * 3 * V;
    for (int x = threadIdx.x; x < 3 * V; x += blockDim.x) {
      const int d = x / V, i = x - d * V;
      const Site s = site_of(i, L);
      Jc[d * V + plane_idx(i, colour_of(s), Vh)] = Jg[x];
    }
    __syncthreads();
    for (int x = threadIdx.x; x < g.NPT; x += blockDim.x) kof[cat[x]] = x % g.NT;
  }
  __syncthreads();
  const uint32_t t = *st.t_dev;
  const int lane = lane_id();
  const int sh = 31 - (lane & 31), hi_shift = lane & 32;
  const FP kNoClone = -__builtin_huge_val();
  // blockDim.x is a multiple of 64, so all lanes of a wave take the same trips
  for (int base = 0; base < g.NPT; base += blockDim.x) {
    const int c = base + static_cast<int>(threadIdx.x);
    const bool active = c < g.NPT;
    const int word = c >> 5;           // this lane's 32-clone word
    const bool write = word < g.NWPT;  // lanes past the last PT word read word base/32 and write nothing
    const uint32_t* P = sp + size_t(write ? word : base >> 5) * V;
    uint32_t* Pw = sp + size_t(write ? word : base >> 5) * V;
    const int cw = active ? c : base;
    int k_cw = 0;  // temperature index of clone cw
    if constexpr (kScalarJ) {
      for (int x = 0; x < g.NPT; ++x) k_cw = cat_g[x] == cw ? x % g.NT : k_cw;
    } else {
      k_cw = kof[cw];
    }
    const double Tk = st.T64[k_cw];
    double* wslot = st.walker + size_t(sample) * g.NPT + cw;
    FP W = active ? static_cast<FP>(*wslot) : kNoClone;
    MicsaRow<H> ra, rb;
    MicsaJ<FP, H> J;
    const RowOff first = row_off<H>(0, 0, L * H, (L - 1) * L * H, 0);  // row 0 of plane 0, colour 0
    micsa_load<H>(ra, P, first);
    if constexpr (!kScalarJ) micsa_load_j<FP, H>(J, Jc, first);
    for (int mm = 0; mm < run.n_pt; ++mm) {
      const int m = run.m_pt0 + mm;
      if (m % g.micsa_refresh == 0) {
        const Block blk = philox10(ctr_word(0, static_cast<uint32_t>(m), kWalker), t, static_cast<uint32_t>(cw),
                                   static_cast<uint32_t>(sample), g.key0, g.key1);
        const uint64_t b53 = ((static_cast<uint64_t>(blk.w1) << 32) | blk.w0) >> 11;
        const FP w = static_cast<FP>(Tk * -log_unit64(static_cast<double>(b53 + 1) * 0x1p-53));
        W = active ? w : kNoClone;
      }
      micsa_half_sweep<FP, H, 0>(ra, rb, J, P, Pw, Jc, sh, hi_shift, write, W);
      micsa_half_sweep<FP, H, 1>(ra, rb, J, P, Pw, Jc, sh, hi_shift, write, W);
    }
    if (active) *wslot = static_cast<double>(W);
  }
  __syncthreads();
  store_spins(g, sp, st, sample, g.NWPT);
}

// LDS of the MicSA kernel: spins and permutation, plus the couplings when
// with_j.
size_t micsa_lds_bytes(const Geo& g, int fp_bytes, bool with_j) {
  const size_t base = align_up(align_up(sizeof(uint32_t) * size_t(g.NWPT) * g.V, 16) +
                                   sizeof(int32_t) * size_t(g.NR * g.NT + g.NPT), 16);
  return base + (with_j ? size_t(fp_bytes) * 3 * g.V : 0);
}

// With P workgroups per sample, part p holds the clone groups j (Philox
// blocks counted from the word's first clone) with j % P == p: the bits
// ((b / G) % P == p) of every word, G clones per block.  Its sweeps touch no
// other bit, and no other part touches these, so each part merges its result
// into the sample's words with an atomic XOR of its own changed bits (the
// global word still holds this part's bits as loaded).
template <typename FP>
__device__ __forceinline__ void store_part(const Geo& g, const uint32_t* sp, const State& st, int sample, int part,
                                           int P, int w_begin, int w_end) {
  constexpr int G = sizeof(FP) == 8 ? 2 : 4;
  uint32_t mask = 0;
  for (int b = 0; b < 32; ++b) mask |= ((b / G) % P == part) ? 1u << b : 0u;
  uint32_t* gsp = st.spins + size_t(sample) * g.NW * g.V;
  const int end = w_end * g.V;
  for (int x = w_begin * g.V + static_cast<int>(threadIdx.x); x < end; x += blockDim.x) {
    const uint32_t change = (sp[x] ^ gsp[x]) & mask;
    if (change) atomicXor(&gsp[x], change);
  }
}

template <typename FP, int CH, bool kSplit, bool kHB>
__global__ __launch_bounds__(kMaxThreads) void sweep_kernel(Geo g, State st, Run run) {
  const int P = run.sample_split;
  const int sample = run.sample_begin + static_cast<int>(blockIdx.x) / P;
  const int part = static_cast<int>(blockIdx.x) % P;
  if (sample >= g.S) return;  // the whole workgroup leaves together
  const Lds s = lds_view(g, sizeof(FP));
  load_spins(g, s, st, sample);
  __syncthreads();
  const FP* Js = static_cast<const FP*>(st.J) + size_t(sample) * 3 * g.V;
  const FP* bc = static_cast<const FP*>(st.beta_clone) + size_t(sample) * g.C;
  const uint32_t t = *st.t_dev;
  // beta of the coldest temperature in the units the clone table holds
  const float beta_cold = sizeof(FP) == 8 ? static_cast<float>(st.beta64[0]) : st.beta32[0];
  sweep_phase<FP, CH, kSplit, kHB>(g, s, Js, bc, sample, t, run.m_pt0, run.n_pt, run.m_er0, run.n_er,
                                   run.early_beta, beta_cold, run.clone_split, part, P);
  // only the words of the clone classes swept here go back: a launch of
  // reservoir sweeps alone may run beside the Houdayer step, which writes the
  // PT words meanwhile (and a launch of PT sweeps alone beside the reservoir's)
  const int w_begin = run.n_pt > 0 ? 0 : g.NWPT;
  const int w_end = run.n_er > 0 && g.NER > 0 ? g.NW : g.NWPT;
  if (P == 1) {
    __syncthreads();
    const size_t stride = size_t(g.NW) * g.V;
    uint32_t* gsp = st.spins + size_t(sample) * stride;
    const size_t b = size_t(w_begin) * g.V, e = size_t(w_end) * g.V;
    if (b % 4 == 0 && e % 4 == 0) {
      const uint4* src = reinterpret_cast<const uint4*>(s.sp + b);
      uint4* dst = reinterpret_cast<uint4*>(gsp + b);
      for (size_t x = threadIdx.x; x < (e - b) / 4; x += blockDim.x) dst[x] = src[x];
    } else {
      for (size_t x = b + threadIdx.x; x < e; x += blockDim.x) gsp[x] = s.sp[x];
    }
  } else {
    __syncthreads();  // every wave's flips are in LDS
    store_part<FP>(g, s.sp, st, sample, part, P, w_begin, w_end);
  }
}

// Houdayer moves (or cluster labels) of one sample per workgroup; the LDS
// layout depends on run.hou_moves, the number of moves labelled at once.
// kLdsRows: the PT spin words are loaded into LDS, read there and flipped
// there; otherwise (samples whose words would keep a CU to one workgroup, in
// launches with more samples than CUs or beside other work; houdayer_plan)
// the overlap rows come from global memory and the flips are collected as
// masks and applied in chunks of run.hou_chunk moves.
template <bool kLdsRows>
__global__ __launch_bounds__(kMaxThreads) void houdayer_kernel(Geo g, State st, Run run) {
  const int sample = run.sample_begin + blockIdx.x;
  if (sample >= g.S) return;
  const bool labels = (run.phases & kPhaseLabels) != 0;
  const bool stats = (run.phases & kPhaseClusterStats) != 0;
  const bool flips = !labels && !stats;
  const int C = flips && !kLdsRows ? run.hou_chunk : 0;
  HouLds s = hou_view(g, run.hou_moves, kLdsRows, stats, C);
  if constexpr (kLdsRows) {
    load_spins(g, s.sp, s.cat, st, sample, g.NWPT);  // Houdayer pairs are PT clones
  } else {
    s.sp = st.spins + size_t(sample) * g.NW * g.V;  // words 0 .. NWPT-1: the PT clones
    for (int x = threadIdx.x; x < g.NR * g.NT; x += blockDim.x) s.cat[x] = st.clone_at[size_t(sample) * g.NR * g.NT + x];
  }
  __syncthreads();
  const bool bad = houdayer_moves<kLdsRows>(g, s, run.hou_moves, C, sample, *st.t_dev, labels ? run.labels : nullptr,
                                            stats ? run.labels : nullptr);
  if constexpr (kLdsRows) {
    if (flips) store_spins(g, s.sp, st, sample, g.NWPT);
  }
  if (bad) atomicOr(&st.status[sample], kStatusUnionBound);
}

template <typename FP, int CH>
__global__ __launch_bounds__(kMaxThreads) void pt_kernel(Geo g, State st, Run run) {
  const int sample = run.sample_begin + blockIdx.x;
  if (sample >= g.S) return;
  const Lds s = lds_view(g, sizeof(FP));
  load_spins(g, s, st, sample);
  for (int x = threadIdx.x; x < g.NR; x += blockDim.x) s.head[x] = st.er_head[size_t(sample) * g.NR + x];
  for (int x = threadIdx.x; x < g.NPT; x += blockDim.x) s.rt[x] = st.rt_state[size_t(sample) * g.NPT + x];
  __syncthreads();
  const FP* beta_fp;
  if constexpr (sizeof(FP) == 8) beta_fp = reinterpret_cast<const FP*>(st.beta64);
  else beta_fp = reinterpret_cast<const FP*>(st.beta32);
  pt_phase<FP, CH>(g, st, sample, *st.t_dev, run.do_reservoir, beta_fp);
  if (run.do_reservoir && g.NERG > 0) store_spins(g, s, st, sample);
  FP* bcg = static_cast<FP*>(st.beta_clone) + size_t(sample) * g.C;
  const FP* bcl = static_cast<const FP*>(s.bcl);
  for (int x = threadIdx.x; x < g.C; x += blockDim.x) bcg[x] = bcl[x];
  for (int x = threadIdx.x; x < g.NR * g.NT; x += blockDim.x) st.clone_at[size_t(sample) * g.NR * g.NT + x] = s.cat[x];
  for (int x = threadIdx.x; x < g.NR; x += blockDim.x) st.er_head[size_t(sample) * g.NR + x] = s.head[x];
  for (int x = threadIdx.x; x < g.NPT; x += blockDim.x) st.rt_state[size_t(sample) * g.NPT + x] = s.rt[x];
}

template <typename FP, int CH>
__global__ __launch_bounds__(kMaxThreads) void measure_kernel(Geo g, State st, Obs ob, Run run) {
  const int sample = run.sample_begin + blockIdx.x;
  if (sample >= g.S) return;
  load_spins(g, lds_view(g, sizeof(FP)), st, sample);
  __syncthreads();
  measure_phase<FP, CH>(g, st, ob, sample, run.meas_k, run.e_current != 0);
}

// Initial spins: bit = sign bit of word 0 of the INIT block of (site, clone).
__global__ void init_kernel(Geo g, State st) {
  const size_t total = size_t(g.S) * g.NW * g.V;
  for (size_t x = blockIdx.x * size_t(blockDim.x) + threadIdx.x; x < total; x += size_t(gridDim.x) * blockDim.x) {
    const int j = static_cast<int>(x % g.V);
    const int w = static_cast<int>((x / g.V) % g.NW);
    const int sample = static_cast<int>(x / (size_t(g.V) * g.NW));
    const int colour = j >= g.Vh;
    const int i0 = 2 * (j - colour * g.Vh);
    const Site s0 = site_of(i0, g.L);
    const int i = i0 + ((s0.y + s0.z + colour) & 1);
    int clone0, nbits;
    if (w < g.NWPT) {
      clone0 = 32 * w;
      nbits = min(32, g.NPT - clone0);
    } else {
      clone0 = g.NPT + 32 * (w - g.NWPT);
      nbits = min(32, g.NPT + g.NER - clone0);
    }
    uint32_t word = 0;
    for (int b = 0; b < nbits; ++b) {
      const Block blk = philox10(ctr_word(i, 0, kInit), 0u, static_cast<uint32_t>(clone0 + b),
                                 static_cast<uint32_t>(sample), g.key0, g.key1);
      word |= (blk.w0 >> 31) << b;
    }
    st.spins[x] = word;
  }
}

// The FP32 couplings again, in the spin words' plane order (the MicSA row
// kernel reads them so through the scalar cache).
__global__ void j_plane_kernel(Geo g, State st) {
  const size_t total = size_t(g.S) * 3 * g.V;
  const float* J = static_cast<const float*>(st.J);
  for (size_t x = blockIdx.x * size_t(blockDim.x) + threadIdx.x; x < total; x += size_t(gridDim.x) * blockDim.x) {
    const int i = static_cast<int>(x % g.V);
    const size_t row = x / g.V;  // sample * 3 + direction
    st.J_plane[row * g.V + plane_idx(i, colour_of(site_of(i, g.L)), g.Vh)] = J[x];
  }
}

// Closes an EMCS: t += 1 (one work-item).
__global__ void advance_t_kernel(uint32_t* t) { *t += 1u; }

__global__ void zero_kernel(uint32_t* p, size_t n) {
  for (size_t x = blockIdx.x * size_t(blockDim.x) + threadIdx.x; x < n; x += size_t(gridDim.x) * blockDim.x) p[x] = 0u;
}

template <typename K>
hipError_t set_lds(K kern, size_t lds) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                             static_cast<int>(lds));
}

template <typename FP, int CH>
hipError_t prepare_t(size_t lds) {
  hipError_t e;
  if ((e = set_lds(sweep_kernel<FP, CH, false, false>, lds)) != hipSuccess) return e;
  if ((e = set_lds(sweep_kernel<FP, CH, true, false>, lds)) != hipSuccess) return e;
  if ((e = set_lds(sweep_kernel<FP, CH, false, true>, lds)) != hipSuccess) return e;
  if ((e = set_lds(sweep_kernel<FP, CH, true, true>, lds)) != hipSuccess) return e;
  if ((e = set_lds(houdayer_kernel<true>, lds)) != hipSuccess) return e;
  if ((e = set_lds(houdayer_kernel<false>, lds)) != hipSuccess) return e;
  if ((e = set_lds(micsa_kernel<FP, true>, lds)) != hipSuccess) return e;
  if ((e = set_lds(micsa_kernel<FP, false>, lds)) != hipSuccess) return e;
  if ((e = set_lds(micsa_row_kernel<FP, 2, false>, lds)) != hipSuccess) return e;
  if constexpr (sizeof(FP) == 4)
    if ((e = set_lds(micsa_row_kernel<FP, 2, true>, lds)) != hipSuccess) return e;
  if ((e = set_lds(micsa_row_kernel<FP, 3, false>, lds)) != hipSuccess) return e;
  if constexpr (sizeof(FP) == 4)
    if ((e = set_lds(micsa_row_kernel<FP, 3, true>, lds)) != hipSuccess) return e;
  if ((e = set_lds(micsa_row_kernel<FP, 4, false>, lds)) != hipSuccess) return e;
  if constexpr (sizeof(FP) == 4)
    if ((e = set_lds(micsa_row_kernel<FP, 4, true>, lds)) != hipSuccess) return e;
  if ((e = set_lds(micsa_row_kernel<FP, 5, false>, lds)) != hipSuccess) return e;
  if constexpr (sizeof(FP) == 4)
    if ((e = set_lds(micsa_row_kernel<FP, 5, true>, lds)) != hipSuccess) return e;
  if ((e = set_lds(micsa_row_kernel<FP, 6, false>, lds)) != hipSuccess) return e;
  if constexpr (sizeof(FP) == 4)
    if ((e = set_lds(micsa_row_kernel<FP, 6, true>, lds)) != hipSuccess) return e;
  if ((e = set_lds(micsa_row_kernel<FP, 7, false>, lds)) != hipSuccess) return e;
  if constexpr (sizeof(FP) == 4)
    if ((e = set_lds(micsa_row_kernel<FP, 7, true>, lds)) != hipSuccess) return e;
  if ((e = set_lds(micsa_row_kernel<FP, 8, false>, lds)) != hipSuccess) return e;
  if constexpr (sizeof(FP) == 4)
    if ((e = set_lds(micsa_row_kernel<FP, 8, true>, lds)) != hipSuccess) return e;
  if ((e = set_lds(pt_kernel<FP, CH>, lds)) != hipSuccess) return e;
  return set_lds(measure_kernel<FP, CH>, lds);
}

template <typename FP, int CH>
hipError_t launch_t(const Geo& g, const State& st, const Obs& ob, const Run& run, const Shape& sh, int n_blocks,
                    hipStream_t stream) {
  const int threads = sh.threads, split = sh.split, parts = sh.parts;
  const size_t lds = plan_lds(g, sizeof(FP)).total;
  hipError_t e = hipSuccess;
  if (run.phases & kPhaseSweep) {
    Run r = run;
    r.clone_split = split;
    if (g.update == kMicsa) {
      // MicSA on the PT clones (one lane per clone), Metropolis on the reservoir
      if (r.n_pt > 0) {
        const int mt = g.NPT >= kMaxThreads ? kMaxThreads : (g.NPT + kWave - 1) / kWave * kWave;
        const bool jl = micsa_lds_bytes(g, sizeof(FP), true) <= kLdsMax;
        auto mk = jl ? micsa_kernel<FP, true> : micsa_kernel<FP, false>;
        int bt = mt;
        size_t lds_m = micsa_lds_bytes(g, sizeof(FP), jl);
        if (jl && g.L >= 4 && g.L <= 16) {
          // the row-wise form (same result); FP32 with the plane-order copy of
          // the couplings reads them through the scalar cache
          bt = mt < kMicsaRowThreads ? mt : kMicsaRowThreads;
          constexpr bool kF32 = sizeof(FP) == 4;
          const bool sj = kF32 && st.J_plane != nullptr;
          if (sj) lds_m = align_up(sizeof(uint32_t) * size_t(g.NWPT) * g.V, 16);
#define PTHR_ROW(HH) (sj ? micsa_row_kernel<FP, HH, kF32> : micsa_row_kernel<FP, HH, false>)
          switch (g.L / 2) {
            case 2: mk = PTHR_ROW(2); break;
            case 3: mk = PTHR_ROW(3); break;
            case 4: mk = PTHR_ROW(4); break;
            case 5: mk = PTHR_ROW(5); break;
            case 6: mk = PTHR_ROW(6); break;
            case 7: mk = PTHR_ROW(7); break;
            default: mk = PTHR_ROW(8); break;
          }
#undef PTHR_ROW
        }
        hipLaunchKernelGGL(mk, dim3(n_blocks), dim3(bt), lds_m, stream, g, st, r);
        if ((e = hipGetLastError()) != hipSuccess) return e;
      }
      r.n_pt = 0;
    }
    if (r.n_pt > 0 || (r.n_er > 0 && g.NER > 0)) {
      r.sample_split = parts;
      const bool shared = split > 1 || parts > 1;  // clone words shared by several waves
      auto k = g.update == kHeatBath
                   ? (shared ? sweep_kernel<FP, CH, true, true> : sweep_kernel<FP, CH, false, true>)
                   : (shared ? sweep_kernel<FP, CH, true, false> : sweep_kernel<FP, CH, false, false>);
      hipLaunchKernelGGL(k, dim3(n_blocks * parts), dim3(threads * split), lds, stream, g, st, r);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  if (run.phases & (kPhaseHoudayer | kPhaseLabels | kPhaseClusterStats)) {
    Run r = run;
    const bool stats = (run.phases & kPhaseClusterStats) != 0;
    const bool flips = (run.phases & (kPhaseLabels | kPhaseClusterStats)) == 0;
    const HouPlan hp = houdayer_plan(g, threads, stats, flips, sh.hou_occupancy != 0);
    if (hp.M < 1) return hipErrorInvalidConfiguration;
    r.hou_moves = hp.M;
    r.hou_chunk = hp.C;
    if (hp.lds_rows) {
      hipLaunchKernelGGL(houdayer_kernel<true>, dim3(n_blocks), dim3(threads), hou_lds_bytes(g, hp.M, true, stats),
                         stream, g, st, r);
    } else {
      // one work-item per row of each move labelled at once
      const int ht = (hp.M * g.L * g.L + kWave - 1) / kWave * kWave;
      hipLaunchKernelGGL(houdayer_kernel<false>, dim3(n_blocks), dim3(ht), hou_lds_bytes(g, hp.M, false, stats, hp.C),
                         stream, g, st, r);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (run.phases & kPhasePT) {
    auto k = pt_kernel<FP, CH>;
    hipLaunchKernelGGL(k, dim3(n_blocks), dim3(threads), lds, stream, g, st, run);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (run.phases & kPhaseMeasure) {
    auto k = measure_kernel<FP, CH>;
    Run r = run;
    r.meas_k = measure_rows_per_pass(g, threads, sizeof(FP));
    const size_t lm = lds + (r.meas_k > 0 ? sizeof(uint32_t) * size_t(r.meas_k) * g.NR * g.L * g.L : 0);
    hipLaunchKernelGGL(k, dim3(n_blocks), dim3(threads), lm, stream, g, st, ob, r);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return e;
}

}  // namespace

// Workspace for the allocation-free autotuner: a copy of the state buffer on
// which candidate schedules run trial EMCS.  Its name is only a host-side
// stand-in for the device array: host code uses the address
// scratch_address returns for the current device, never the name.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(void** ptr) { return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch)); }

size_t lds_bytes(const Geo& g, int fp_bytes) {
  const size_t phases = plan_lds(g, fp_bytes).total, hou = hou_lds_bytes(g, 1, true);
  return phases > hou ? phases : hou;
}

// Temperatures whose overlaps are taken at once by the row-parallel form: one
// x-row per work-item and the clones' row masks in LDS after the phase plan;
// 0 selects the per-site form.
int measure_rows_per_pass(const Geo& g, int threads, int fp_bytes) {
  const size_t base = plan_lds(g, fp_bytes).total, per_k = sizeof(uint32_t) * size_t(g.NR) * g.L * g.L;
  int KC = threads / (g.L * g.L);
  if (KC > g.NT) KC = g.NT;
  while (KC > 0 && base + per_k * KC > kLdsMax) --KC;
  return KC;
}

// Houdayer moves labelled at once: one x-row per work-item, as many moves as
// the workgroup has rows for and LDS holds (at least one: a workgroup has at
// least V/8 >= L^2 work-items, rounded up to whole waves); the launch takes
// M L^2 work-items.
bool micsa_scalar_couplings(int L, int NWPT, int n_cat, int NPT) {
  (void)n_cat;
  (void)NPT;
  if (L < 4 || L > 16) return false;  // the row kernel's sizes
  const size_t V = size_t(L) * L * L;
  const size_t spins = align_up(sizeof(uint32_t) * size_t(NWPT) * V, 16);
  return 2 * spins <= kLdsMax;
}

HouPlan houdayer_plan(const Geo& g, int threads, bool stats, bool flips, bool occupancy) {
  const int n_moves = hou_moves(g);
  int cap = threads / (g.L * g.L);
  if (cap > n_moves) cap = n_moves;
  if (cap > kMaxHouMoves) cap = kMaxHouMoves;
  // spin words in LDS: as many moves as the workgroup has rows for and LDS holds
  int M = cap;
  while (M > 0 && hou_lds_bytes(g, M, true, stats) > kLdsMax) --M;
  // (rows read four words at a time, L % 8 == 0; flips applied one row of
  // at most 16 sites per work-item, L <= 16)
  if (M == 0 || !flips || !occupancy || g.L % 8 != 0 || g.L > 16 ||
      2 * hou_lds_bytes(g, M, true, stats) <= kLdsMax)
    return HouPlan{M, 0, true};
  // The words keep a CU to one workgroup: with the rows read from global
  // memory (four words at a time) and every flip collected before one
  // application, two workgroups share a CU where LDS allows it and they label
  // at least as many moves together (the kernel waits on LDS latency, so more
  // waves per CU pay).
  int M2 = cap;
  auto all = [&](int m) { return (n_moves + m - 1) / m * m; };
  while (M2 > 0 && hou_lds_bytes(g, M2, false, stats, all(M2)) > kLdsMax / 2) --M2;
  if (M2 > 0 && 2 * M2 >= M) return HouPlan{M2, all(M2), false};
  return HouPlan{M, 0, true};
}

hipError_t launch_emcs(int precision, const Geo& g, const State& st, const Obs& ob, const Run& run,
                       const Shape& sh, int n_blocks, hipStream_t stream) {
#define PTHR_LAUNCH(FP, CH) \
  return launch_t<FP, CH>(g, st, ob, run, sh, n_blocks, stream)
  if (precision == 0) {
    switch (sh.chunk) {
      case 2: PTHR_LAUNCH(double, 2);
      case 4: PTHR_LAUNCH(double, 4);
    }
  } else {
    switch (sh.chunk) {
      case 2: PTHR_LAUNCH(float, 2);
      case 4: PTHR_LAUNCH(float, 4);
      case 8: PTHR_LAUNCH(float, 8);
    }
  }
#undef PTHR_LAUNCH
  return hipErrorInvalidValue;
}

hipError_t prepare_kernels(size_t lds) {
  hipError_t e;
  if ((e = prepare_t<double, 2>(lds)) != hipSuccess) return e;
  if ((e = prepare_t<double, 4>(lds)) != hipSuccess) return e;
  if ((e = prepare_t<float, 2>(lds)) != hipSuccess) return e;
  if ((e = prepare_t<float, 4>(lds)) != hipSuccess) return e;
  return prepare_t<float, 8>(lds);
}

hipError_t launch_advance_t(const State& st, hipStream_t stream) {
  hipLaunchKernelGGL(advance_t_kernel, dim3(1), dim3(1), 0, stream, st.t_dev);
  return hipGetLastError();
}

hipError_t launch_init(const Geo& g, const State& st, hipStream_t stream) {
  const size_t total = size_t(g.S) * g.NW * g.V;
  const int threads = 256;
  const int blocks = static_cast<int>((total + threads - 1) / threads < 65536 ? (total + threads - 1) / threads : 65536);
  hipLaunchKernelGGL(init_kernel, dim3(blocks), dim3(threads), 0, stream, g, st);
  if (st.J_plane) {
    const size_t nj = size_t(g.S) * 3 * g.V;
    const int bj = static_cast<int>((nj + threads - 1) / threads < 65536 ? (nj + threads - 1) / threads : 65536);
    hipLaunchKernelGGL(j_plane_kernel, dim3(bj), dim3(threads), 0, stream, g, st);
  }
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t stream) {
  const size_t n = bytes / 4;
  if (n == 0) return hipSuccess;
  const int threads = 256;
  const int blocks = static_cast<int>((n + threads - 1) / threads < 4096 ? (n + threads - 1) / threads : 4096);
  hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(threads), 0, stream, static_cast<uint32_t*>(p), n);
  return hipGetLastError();
}

}  // namespace pthr
