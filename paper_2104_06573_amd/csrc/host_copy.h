// Library-internal (not part of the C ABI): a call's results copied to
// pinned host memory by one kernel on the call's stream, which reads the
// track count on the device -- the server's lanes use it so that a batch
// needs no host round trip between its reconstruction and the copy of
// exactly the tracks found.
#pragma once

#include <hip/hip_runtime.h>

#include "pxt.h"

namespace pxt {

// Pinned host destinations (device-accessible host memory), each with room
// for the capacity of the call's pxt_tracks.
struct HostTracks {
  uint32_t* hit_idx;  // [capacity][8]
  uint8_t* n_hits;    // [capacity]
  float* params;      // [capacity][5]
  float* cov;         // [capacity][15]
  float* chi2;        // [capacity][2]
  uint8_t* flags;     // [capacity]
  uint32_t* per_event_tracks;  // [n_events]
  pxt_counts* counts;          // [1]
};

// Enqueues the copy on stream s after the call's work: counts and
// per-event track counts always, the tracks' arrays for the n_tracks of
// the counts when their status is PXT_OK.  dev holds the call's device
// outputs (as passed to pxt_reconstruct).
hipError_t launch_copy_out(const pxt_tracks& dev, uint32_t n_events, const HostTracks& host,
                           hipStream_t s);

}  // namespace pxt
