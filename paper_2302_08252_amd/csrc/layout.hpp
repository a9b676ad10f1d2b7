// layout.hpp -- record layouts of the track buffers and the field accessor.
//
// A track record has 14 fields ("leaves"), in this order:
//   0-2 pos (f64)   3-5 dir   6 E   7 numIALeft   8 trackId (u64)   9 parentId (u64)
//   10 rngSeed (u32)   11 rngCtr (u32)   12 volume (i32)   13 event (u32)
// dir, E and numIALeft are f64 in the FP64 record (96 bytes, no padding) and
// f32 in the mixed record (76 bytes of data; the AoS stride is 80 with 4 bytes
// of padding after numIALeft so that trackId stays 8-aligned).
//
// Mappings (paper Sec. 3-4, the layouts the paper switches between):
//   AoS      addr = slot * stride + offset(leaf)
//   SoA      addr = start(leaf) + slot * size(leaf), each field array 256-byte aligned
//   AoSoA-N  addr = (slot / N) * N * R + N * prefix(leaf) + (slot % N) * size(leaf),
//            N a power of two in [2, 256], R the unpadded record size
//            (paper Sec. 4: fields (A,B,C) with N = 2 are laid out AABBCCAABBCC)
//   per type one of the three above for each particle type's buffers (the per-
//            particle-type layouts proposed as future work in paper Sec. 6), all
//            written as addr = (slot >> g) * B + F(leaf) + (slot & (2^g - 1)) * size(leaf):
//            AoS g = 0, B = stride, F = offset; SoA g = 63, F = start;
//            AoSoA-N g = log2 N, B = N * R, F = N * prefix
//
// The accessor routes every field load and store through the mapping; its
// instrumented form (paper Sec. 5) counts reads and writes per field (one
// atomic per wavefront, access site and counter) and every access per 4-byte word of
// the buffer, indexed by the actual byte address (a per-byte heatmap at 1/4 of
// the memory, exact because every field is a multiple of 4 bytes).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Streaming (non-temporal) loads and stores of track fields: every field is
// read once and written once per iteration, far beyond the caches' reach.
#ifndef ADEPT_NT
#define ADEPT_NT 0
#endif

namespace adept {

enum : int { MAP_AOS = 0, MAP_SOA = 1, MAP_AOSOA = 2, MAP_TYPED = 3 };
enum : int { SPARSE = 0, DENSE = 1 };

template <bool MIXED>
struct Rec;

template <>
struct Rec<false> {
  static constexpr uint32_t stride = 96, bytes = 96;
  __host__ __device__ static constexpr uint32_t size(int l) { return l < 10 ? 8u : 4u; }
  __host__ __device__ static constexpr uint32_t off(int l) { return l < 10 ? 8u * l : 80u + 4u * (l - 10); }
  __host__ __device__ static constexpr uint32_t prefix(int l) { return off(l); }
  // 4-byte and 8-byte fields before field l (SoA start offsets)
  __host__ __device__ static constexpr uint32_t n4(int l) { return l <= 10 ? 0u : (uint32_t)(l - 10); }
  __host__ __device__ static constexpr uint32_t n8(int l) { return l < 10 ? (uint32_t)l : 10u; }
};

template <>
struct Rec<true> {
  static constexpr uint32_t stride = 80, bytes = 76;
  __host__ __device__ static constexpr uint32_t size(int l) {
    return (l < 3 || l == 8 || l == 9) ? 8u : 4u;
  }
  // AoS offsets: pos 0..16, dir 24..32, E 36, numIALeft 40, pad 44, ids 48, 56, u32s 64..76
  __host__ __device__ static constexpr uint32_t off(int l) {
    return l < 3 ? 8u * l : (l < 8 ? 24u + 4u * (l - 3) : (l < 10 ? 48u + 8u * (l - 8) : 64u + 4u * (l - 10)));
  }
  // unpadded prefix sums (AoSoA)
  __host__ __device__ static constexpr uint32_t prefix(int l) {
    return l < 3 ? 8u * l : (l < 8 ? 24u + 4u * (l - 3) : (l < 10 ? 44u + 8u * (l - 8) : 60u + 4u * (l - 10)));
  }
  // 4-byte and 8-byte fields before field l (SoA start offsets)
  __host__ __device__ static constexpr uint32_t n4(int l) {
    return l <= 3 ? 0u : (l <= 8 ? (uint32_t)(l - 3) : (l <= 10 ? 5u : 5u + (uint32_t)(l - 10)));
  }
  __host__ __device__ static constexpr uint32_t n8(int l) { return l <= 3 ? (uint32_t)l : (l <= 8 ? 3u : (l <= 10 ? 3u + (uint32_t)(l - 8) : 5u)); }
};

// Runtime parameters of one mapping instance (host-computed, passed by value).
struct MapArgs {
  uint64_t soa_start[14];  // SoA: byte offset of each field array; per type: F(leaf)
  uint64_t a4, a8;         // SoA: the padded sizes of a 4-byte and of an 8-byte field array
                           // (soa_start[l] = n4(l) * a4 + n8(l) * a8)
  uint32_t lg;             // AoSoA: log2 N; per type: g
  uint32_t pad;
  uint64_t blk;            // per type: B
};

__host__ __device__ inline uint64_t align256(uint64_t x) { return (x + 255u) & ~(uint64_t)255u; }

template <bool MIXED>
inline MapArgs make_map_args(int map, uint32_t lanes, uint64_t C) {
  MapArgs m{};
  uint64_t a = 0;
  for (int l = 0; l < 14; ++l) {
    m.soa_start[l] = a;
    a = align256(a + C * Rec<MIXED>::size(l));
  }
  m.a4 = align256(4 * C);
  m.a8 = align256(8 * C);
  uint32_t lg = 0;
  while ((1u << lg) < lanes) ++lg;
  m.lg = map == MAP_AOSOA ? lg : 0;
  return m;
}

// The per-type form of mapping `map` (AoS, SoA or AoSoA with `lanes` lanes).
template <bool MIXED>
inline MapArgs make_typed_args(int map, uint32_t lanes, uint64_t C) {
  using RC = Rec<MIXED>;
  MapArgs m = make_map_args<MIXED>(map, lanes, C);
  if (map == MAP_AOS) {
    m.lg = 0;
    m.blk = RC::stride;
    for (int l = 0; l < 14; ++l) m.soa_start[l] = RC::off(l);
  } else if (map == MAP_SOA) {
    m.lg = 63;
    m.blk = 0;
  } else {
    m.blk = (uint64_t)lanes * RC::bytes;
    for (int l = 0; l < 14; ++l) m.soa_start[l] = (uint64_t)RC::prefix(l) << m.lg;
  }
  return m;
}

template <bool MIXED>
inline uint64_t buffer_bytes(int map, uint32_t lanes, uint64_t C) {
  (void)lanes;
  if (map == MAP_AOS) return C * Rec<MIXED>::stride;
  if (map == MAP_SOA) {
    uint64_t a = 0;
    for (int l = 0; l < 14; ++l) a = align256(a + C * Rec<MIXED>::size(l));
    return a;
  }
  return C * Rec<MIXED>::bytes;
}

template <int MAP, bool MIXED>
__host__ __device__ __forceinline__ uint64_t leaf_addr(const MapArgs& m, uint64_t slot, int l) {
  using RC = Rec<MIXED>;
  if (MAP == MAP_AOS) return slot * RC::stride + RC::off(l);
  // two scalars instead of fourteen start offsets (the same values: field arrays
  // start 256-aligned, so each one's padded size is align256(C * size))
  if (MAP == MAP_SOA) return RC::n4(l) * m.a4 + RC::n8(l) * m.a8 + slot * RC::size(l);
  if (MAP == MAP_TYPED)
    return (slot >> m.lg) * m.blk + m.soa_start[l] + (slot & ((1ull << m.lg) - 1)) * RC::size(l);
  const uint64_t mask = (1ull << m.lg) - 1;
  return (slot & ~mask) * RC::bytes + ((uint64_t)RC::prefix(l) << m.lg) + (slot & mask) * RC::size(l);
}

// Per-(type, physical buffer) instrumentation counters.
struct Instr {
  unsigned long long* rw;  // [14][2]: reads, writes
  uint32_t* heat;          // one counter per 4-byte word of the buffer
};

template <int MAP, bool MIXED, bool INSTR>
struct Acc {
  uint8_t* base;
  MapArgs m;
  Instr in;
  bool on;  // counting window open

  // Lanes of one wavefront may reach the same access site for different buffers
  // (e.g. creations of different particle types), so the per-field totals are
  // aggregated per distinct counter: one atomic per counter and site.
  __device__ __forceinline__ void count(uint64_t a, int l, int w) const {
    if (INSTR && on) {
      unsigned long long* target = &in.rw[l * 2 + w];
      unsigned long long pending = __ballot(1);
      while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const unsigned long long lead_ptr = __shfl((unsigned long long)(uintptr_t)target, leader, 64);
        const unsigned long long same = __ballot((unsigned long long)(uintptr_t)target == lead_ptr);
        if ((int)__lane_id() == leader) atomicAdd(target, (unsigned long long)__popcll(same));
        pending &= ~same;
      }
      const uint32_t words = Rec<MIXED>::size(l) / 4;
      for (uint32_t k = 0; k < words; ++k) atomicAdd(&in.heat[a / 4 + k], 1u);
    }
  }
  template <class T>
  __device__ __forceinline__ T ld(uint64_t slot, int l) const {
    const uint64_t a = leaf_addr<MAP, MIXED>(m, slot, l);
    count(a, l, 0);
    if (ADEPT_NT) return __builtin_nontemporal_load(reinterpret_cast<const T*>(base + a));
    return *reinterpret_cast<const T*>(base + a);
  }
  template <class T>
  __device__ __forceinline__ void st(uint64_t slot, int l, T v) const {
    const uint64_t a = leaf_addr<MAP, MIXED>(m, slot, l);
    count(a, l, 1);
    if (ADEPT_NT) __builtin_nontemporal_store(v, reinterpret_cast<T*>(base + a));
    else *reinterpret_cast<T*>(base + a) = v;
  }
};

}  // namespace adept
