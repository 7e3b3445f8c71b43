// instantiate.hpp -- builds the launch table of one storage precision.
#pragma once

#include "kernels.hpp"

namespace lbm {

template <int A, int L, int P, int K, int C>
void launch_update(const KArgs &a, uint32_t blocks, hipStream_t s)
{
    hipLaunchKernelGGL((k_update<A, L, P, K, C>), dim3(blocks), dim3(BLOCK), a.lds_bytes, s, a);
}
template <int P, int K, int C>
void launch_pair(const KArgs &a, uint32_t blocks, hipStream_t s)
{
    hipLaunchKernelGGL((k_update_pair<P, K, C>), dim3(blocks), dim3(BLOCK), a.lds_bytes, s, a);
}
template <int P, int K, int C, int L>
void launch_gen(const KArgs &a, uint32_t blocks, hipStream_t s)
{
    hipLaunchKernelGGL((k_update_gen<P, K, C, L>), dim3(blocks), dim3(BLOCK), a.lds_bytes, s, a);
}
template <int P, int K, int C>
void launch_pair_wide(const KArgs &a, uint32_t blocks, hipStream_t s)
{
    hipLaunchKernelGGL((k_update_pair_wide<P, K, C>), dim3(blocks), dim3(BLOCK), a.lds_bytes, s, a);
}
template <int P, int K, int C, int L>
void launch_wide(const KArgs &a, uint32_t blocks, hipStream_t s)
{
    hipLaunchKernelGGL((k_update_wide<P, K, C, L>), dim3(blocks), dim3(BLOCK), a.lds_bytes, s, a);
}
template <int A, int L, int P, int R>
void launch_get(const KArgs &a, uint32_t blocks, hipStream_t s)
{
    hipLaunchKernelGGL((k_get<A, L, P, R>), dim3(blocks), dim3(BLOCK), 0, s, a);
}
template <int A, int L, int P, int R>
void launch_set(const KArgs &a, uint32_t blocks, hipStream_t s)
{
    hipLaunchKernelGGL((k_set<A, L, P, R>), dim3(blocks), dim3(BLOCK), 0, s, a);
}
template <int A, int L, int P, int R>
void launch_init(const KArgs &a, uint32_t blocks, hipStream_t s)
{
    hipLaunchKernelGGL((k_init<A, L, P, R>), dim3(blocks), dim3(BLOCK), 0, s, a);
}
template <int A, int L, int P, int R>
void launch_reduce(const KArgs &a, uint32_t blocks, hipStream_t s)
{
    hipLaunchKernelGGL((k_reduce<A, L, P, R>), dim3(blocks), dim3(BLOCK), 0, s, a);
}

template <int A, int L, int P, int C>
void fill_updates(PrecTable &t)
{
    t.update[A][L][C][K_TS_COLLIDE] = &launch_update<A, L, P, K_TS_COLLIDE, C>;
    t.update[A][L][C][K_TS_STREAM] = &launch_update<A, L, P, K_TS_STREAM, 0>; // no collision
    t.update[A][L][C][K_OS_PUSH] = &launch_update<A, L, P, K_OS_PUSH, C>;
    t.update[A][L][C][K_OS_PULL] = &launch_update<A, L, P, K_OS_PULL, C>;
    t.update[A][L][C][K_AA_EVEN] = &launch_update<A, L, P, K_AA_EVEN, C>;
    t.update[A][L][C][K_AA_ODD] = &launch_update<A, L, P, K_AA_ODD, C>;
    t.update[A][L][C][K_ET0] = &launch_update<A, L, P, K_ET0, C>;
    t.update[A][L][C][K_ET1] = &launch_update<A, L, P, K_ET1, C>;
}

template <int P, int C>
void fill_pairs(PrecTable &t)
{
    t.pair[C][K_TS_COLLIDE] = &launch_pair<P, K_TS_COLLIDE, C>;
    t.pair[C][K_TS_STREAM] = &launch_pair<P, K_TS_STREAM, 0>; // no collision
    t.pair[C][K_OS_PUSH] = &launch_pair<P, K_OS_PUSH, C>;
    t.pair[C][K_OS_PULL] = &launch_pair<P, K_OS_PULL, C>;
    t.pair[C][K_AA_EVEN] = &launch_pair<P, K_AA_EVEN, C>;
    t.pair[C][K_AA_ODD] = &launch_pair<P, K_AA_ODD, C>;
    t.pair[C][K_ET0] = &launch_pair<P, K_ET0, C>;
    t.pair[C][K_ET1] = &launch_pair<P, K_ET1, C>;
}

template <int P, int C, int L>
void fill_gen(PrecTable &t)
{
    t.gen[L == L_BLK][C][K_TS_COLLIDE] = &launch_gen<P, K_TS_COLLIDE, C, L>;
    t.gen[L == L_BLK][C][K_TS_STREAM] = &launch_gen<P, K_TS_STREAM, 0, L>; // no collision
    t.gen[L == L_BLK][C][K_OS_PUSH] = &launch_gen<P, K_OS_PUSH, C, L>;
    t.gen[L == L_BLK][C][K_OS_PULL] = &launch_gen<P, K_OS_PULL, C, L>;
    t.gen[L == L_BLK][C][K_AA_EVEN] = &launch_gen<P, K_AA_EVEN, C, L>;
    t.gen[L == L_BLK][C][K_AA_ODD] = &launch_gen<P, K_AA_ODD, C, L>;
    t.gen[L == L_BLK][C][K_ET0] = &launch_gen<P, K_ET0, C, L>;
    t.gen[L == L_BLK][C][K_ET1] = &launch_gen<P, K_ET1, C, L>;
}

template <int P, int C>
void fill_pairs_wide(PrecTable &t)
{
    t.pair_wide[C][K_TS_COLLIDE] = &launch_pair_wide<P, K_TS_COLLIDE, C>;
    t.pair_wide[C][K_TS_STREAM] = &launch_pair_wide<P, K_TS_STREAM, 0>; // no collision
    t.pair_wide[C][K_OS_PUSH] = &launch_pair_wide<P, K_OS_PUSH, C>;
    t.pair_wide[C][K_OS_PULL] = &launch_pair_wide<P, K_OS_PULL, C>;
    t.pair_wide[C][K_AA_EVEN] = &launch_pair_wide<P, K_AA_EVEN, C>;
    t.pair_wide[C][K_AA_ODD] = &launch_pair_wide<P, K_AA_ODD, C>;
    t.pair_wide[C][K_ET0] = &launch_pair_wide<P, K_ET0, C>;
    t.pair_wide[C][K_ET1] = &launch_pair_wide<P, K_ET1, C>;
}

template <int P, int C, int L>
void fill_wide(PrecTable &t)
{
    t.wide[L == L_BLK][C][K_TS_COLLIDE] = &launch_wide<P, K_TS_COLLIDE, C, L>;
    t.wide[L == L_BLK][C][K_TS_STREAM] = &launch_wide<P, K_TS_STREAM, 0, L>; // no collision
    t.wide[L == L_BLK][C][K_OS_PUSH] = &launch_wide<P, K_OS_PUSH, C, L>;
    t.wide[L == L_BLK][C][K_OS_PULL] = &launch_wide<P, K_OS_PULL, C, L>;
    t.wide[L == L_BLK][C][K_AA_EVEN] = &launch_wide<P, K_AA_EVEN, C, L>;
    t.wide[L == L_BLK][C][K_AA_ODD] = &launch_wide<P, K_AA_ODD, C, L>;
    t.wide[L == L_BLK][C][K_ET0] = &launch_wide<P, K_ET0, C, L>;
    t.wide[L == L_BLK][C][K_ET1] = &launch_wide<P, K_ET1, C, L>;
}

template <int A, int L, int P, int R>
void fill_map(PrecTable &t)
{
    t.get[A][L][R] = &launch_get<A, L, P, R>;
    t.set[A][L][R] = &launch_set<A, L, P, R>;
    t.init[A][L][R] = &launch_init<A, L, P, R>;
    t.reduce[A][L][R] = &launch_reduce<A, L, P, R>;
}

template <int A, int L, int P>
void fill_al(PrecTable &t)
{
    fill_updates<A, L, P, 0>(t);
    fill_updates<A, L, P, 1>(t);
    fill_map<A, L, P, R_LOCAL>(t);
    fill_map<A, L, P, R_PULL>(t);
    fill_map<A, L, P, R_AAODD>(t);
    fill_map<A, L, P, R_ET0>(t);
    fill_map<A, L, P, R_ET1>(t);
}

template <int P>
PrecTable make_table()
{
    PrecTable t{};
    fill_al<A_DIRECT, L_SOA, P>(t);
    fill_pairs<P, 0>(t);
    fill_pairs<P, 1>(t);
    fill_wide<P, 0, L_SOA>(t);
    fill_wide<P, 1, L_SOA>(t);
    fill_wide<P, 0, L_BLK>(t);
    fill_wide<P, 1, L_BLK>(t);
    fill_pairs_wide<P, 0>(t);
    fill_pairs_wide<P, 1>(t);
    fill_gen<P, 0, L_SOA>(t);
    fill_gen<P, 1, L_SOA>(t);
    fill_gen<P, 0, L_BLK>(t);
    fill_gen<P, 1, L_BLK>(t);
    fill_al<A_DIRECT, L_AOS, P>(t);
    fill_al<A_DIRECT, L_BLK, P>(t);
    fill_al<A_INDIRECT, L_SOA, P>(t);
    fill_al<A_INDIRECT, L_AOS, P>(t);
    fill_al<A_INDIRECT, L_BLK, P>(t);
    return t;
}

} // namespace lbm
