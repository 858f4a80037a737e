// host_hash.hpp -- the host side of the hashing path.
//
// The paper computes the last step of direct hashing on the CPU: once the
// segment digests are back from the GPU, the host hashes that buffer into
// the final value (Sec. 3.2.2).  That step is one sequential Merkle-Damgard
// chain, which a CPU core runs many times faster than one GPU lane.  This
// module holds the library's sequential MD5 / SHA-1 for the host (SHA-1 uses
// the processor's SHA instructions where it has them) and a fixed pool of
// host threads that runs several such chains at once.
#pragma once

#include <stdint.h>

#include <functional>

namespace hg {
namespace host {

// Standard digest of p[0, n): 16 bytes for kind 0 (MD5), 20 for kind 1
// (SHA-1), written to out.  Unknown kinds write nothing.
void digest(int kind, const uint8_t *p, uint64_t n, uint8_t *out);

// True when SHA-1 runs on the processor's SHA extensions (x86 SHA-NI);
// HG_HOST_SHA1_PORTABLE in the environment at load time selects the
// portable code instead.
bool sha1_accelerated();

// Runs fn(i) for every i in [0, n) on the pool's threads and the calling
// thread, and returns when all have finished.  Several callers may use the
// pool at once; indices are handed out in ascending order, so callers list
// the longest work first.
void parallel_for(uint64_t n, const std::function<void(uint64_t)> &fn);

// Threads of the pool (besides the callers).
int pool_threads();

}  // namespace host
}  // namespace hg
