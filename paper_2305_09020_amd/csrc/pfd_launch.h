// Kernel launch layer: every kernel of the step is a device body NAME_run(const VGrid& vg, args...)
// with a descriptor struct NAME : KDef<&NAME_run, launch bound, waves per EU>, launched through
// Kern<NAME>::launch.  The body reads its work-group index and grid size from vg, not from the
// hardware registers, so one body serves two kernels:
//  * k_single: one instance, vg = the hardware block index and grid (the ordinary launch);
//  * k_multi: many instances in one launch.  Each instance keeps its own grid, argument list and
//    buffers; the launch's work-groups are the concatenation of all instances' work-groups, and
//    a table maps a work-group to (instance, local index).
// While a context records (ctx->rec set), Kern<...>::launch appends the launch (its multi-instance
// kernel, grid, block, dynamic LDS and packed arguments) to the record instead of issuing it; a
// batch of contexts records one step of each and issues the k_multi launches (pfd_batch.cpp).
#pragma once

#include <cstring>
#include <type_traits>
#include <utility>

#include "pfd_internal.h"

namespace pfd {

struct U3 {
  unsigned x, y, z;
};
// virtual launch coordinates of one work-group: block index b within its instance's grid g.  A
// body maps b to its tile exactly as in a single launch (the XCD-aware remaps included), so an
// instance computes the same tiles, partial sums and results in either kind of launch.
struct VGrid {
  U3 b, g;
};

template <auto F, int LB_, int WPE_>
struct KDef {
  static constexpr auto run = F;
  static constexpr int LB = LB_ > 0 ? LB_ : 1024;   // 1024: the default flat work-group bound
  static constexpr int WPE = WPE_;                   // 0: no waves-per-EU request
};

// argument pack with one layout on host and device (trivially copyable members)
template <class... A>
struct Tup {};
template <class H, class... T>
struct Tup<H, T...> {
  H h;
  Tup<T...> t;
  __host__ __device__ Tup() {}
  __host__ __device__ Tup(H h_, T... t_) : h(h_), t(t_...) {}
};
template <size_t I, class H, class... T>
__host__ __device__ __forceinline__ const auto& tget(const Tup<H, T...>& t) {
  if constexpr (I == 0)
    return t.h;
  else
    return tget<I - 1>(t.t);
}
template <auto F, class P, size_t... I>
__device__ __forceinline__ void tcall(const VGrid& vg, const P& p, std::index_sequence<I...>) {
  F(vg, tget<I>(p)...);
}

// one member of a multi-instance launch: its grid and the first global work-group index
struct MEnt {
  unsigned gx, gy, gz, b0;
};

__device__ __forceinline__ VGrid vg_hw() {
  return VGrid{{blockIdx.x, blockIdx.y, blockIdx.z}, {gridDim.x, gridDim.y, gridDim.z}};
}
// multi-instance work-group: the hardware hands work-groups to the eight XCDs in turn, so the
// global index is first remapped to make each XCD take one contiguous range (the work-groups of
// a small instance then share one L2), then looked up in the table
__device__ __forceinline__ VGrid vg_multi(unsigned total, const unsigned* __restrict__ tab,
                                          const MEnt* __restrict__ ent, unsigned& inst) {
  const unsigned q = total >> 3, r = total & 7, x = blockIdx.x & 7, j = blockIdx.x >> 3;
  const unsigned L = x < r ? x * (q + 1) + j : r * (q + 1) + (x - r) * q + j;
  inst = tab[L];
  const MEnt m = ent[inst];
  const unsigned l = L - m.b0, gxy = m.gx * m.gy, z = l / gxy, rem = l - z * gxy, y = rem / m.gx;
  return VGrid{{rem - y * m.gx, y, z}, {m.gx, m.gy, m.gz}};
}

template <class S, class... A>
__global__ void __launch_bounds__(S::LB) k_single(A... a) {
  S::run(vg_hw(), a...);
}
template <class S, class... A>
__global__ void __launch_bounds__(S::LB) __attribute__((amdgpu_waves_per_eu(S::WPE > 0 ? S::WPE : 1)))
k_single_w(A... a) {
  S::run(vg_hw(), a...);
}
template <class S, class... A>
__global__ void __launch_bounds__(S::LB) k_multi(unsigned total, const unsigned* __restrict__ tab,
                                                 const MEnt* __restrict__ ent, const Tup<A...>* __restrict__ args) {
  unsigned i;
  const VGrid vg = vg_multi(total, tab, ent, i);
  tcall<S::run>(vg, args[i], std::index_sequence_for<A...>{});
}
template <class S, class... A>
__global__ void __launch_bounds__(S::LB) __attribute__((amdgpu_waves_per_eu(S::WPE > 0 ? S::WPE : 1)))
k_multi_w(unsigned total, const unsigned* __restrict__ tab, const MEnt* __restrict__ ent,
          const Tup<A...>* __restrict__ args) {
  unsigned i;
  const VGrid vg = vg_multi(total, tab, ent, i);
  tcall<S::run>(vg, args[i], std::index_sequence_for<A...>{});
}

template <class S, class F = std::remove_cv_t<decltype(S::run)>>
struct Kern;
template <class S, class... A>
struct Kern<S, void (*)(const VGrid&, A...)> {
  static const void* single() {
    if constexpr (S::WPE > 0)
      return reinterpret_cast<const void*>(&k_single_w<S, A...>);
    else
      return reinterpret_cast<const void*>(&k_single<S, A...>);
  }
  static const void* multi() {
    if constexpr (S::WPE > 0)
      return reinterpret_cast<const void*>(&k_multi_w<S, A...>);
    else
      return reinterpret_cast<const void*>(&k_multi<S, A...>);
  }
  // cls >= 0: timing scope of that class (pfd_profile_read); -1: the caller times it
  static void launch(pfd_ctx* c, int cls, dim3 grid, dim3 block, size_t shm, hipStream_t s, A... a) {
    if (c->rec) {
      RecLaunch r;
      r.fn = multi();
      r.grid[0] = grid.x, r.grid[1] = grid.y, r.grid[2] = grid.z;
      r.block[0] = block.x, r.block[1] = block.y, r.block[2] = block.z;
      r.shm = shm;
      const Tup<A...> p(a...);
      r.asize = sizeof(p);
      r.aalign = alignof(Tup<A...>);
      r.args.resize(sizeof(p));
      std::memcpy(r.args.data(), &p, sizeof(p));
      c->rec->push_back(std::move(r));
      return;
    }
    ProfScope ps(cls >= 0 ? c : nullptr, cls);
    if constexpr (S::WPE > 0)
      hipLaunchKernelGGL((k_single_w<S, A...>), grid, block, shm, s, a...);
    else
      hipLaunchKernelGGL((k_single<S, A...>), grid, block, shm, s, a...);
  }
};

}  // namespace pfd
