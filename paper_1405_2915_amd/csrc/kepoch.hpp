// Device side of the descriptor epoch kept in a stream workspace's sync area.
//
// Every workgroup of a call that hands values to other workgroups through
// tagged words reads the epoch when it starts; the last workgroup of the call
// to finish advances it, so the next call (in stream order, or the next
// replay of a captured graph) tags with a new epoch and never mistakes an
// earlier call's words for its own.
#pragma once

#include "kcommon.hpp"
#include "launch.hpp"

namespace skel {
namespace dev {

__device__ __forceinline__ uint32_t epoch_of_call(u64* sync) {
    return (uint32_t)(tag_load(sync + SYNC_EPOCH) % kEpochMax) + 1;
}

__device__ __forceinline__ void epoch_advance(u64* sync) {
    atomicAdd(sync + SYNC_EPOCH, 1ull);
}

}  // namespace dev
}  // namespace skel
