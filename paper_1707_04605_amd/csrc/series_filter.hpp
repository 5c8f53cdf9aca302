// Causal convolution of many equal-length series with one kernel, split in two: the
// constructor does every allocation and host round trip (the kernel's spectrum, the padded
// chunk buffer, the transform plans), enqueue() only launches work on the stream it is
// given.  A caller can thus run the filter of one batch on a stream of its own while
// another stream steps the next batch.
#pragma once

#include <memory>
#include <vector>

#include "mgrt_internal.hpp"

namespace mgrt {

class SeriesFilter {
  public:
    // x of enqueue() holds n_series rows of N samples of FP32 (prec 32) or FP64 (prec 64);
    // h holds N samples.  The transforms are FP64 whatever prec is; scratch_cap bounds the
    // padded chunk buffer (at least one row).
    SeriesFilter(Ctx &c, int prec, int64_t n_series, int64_t N, const std::vector<double> &h,
                 size_t scratch_cap);
    ~SeriesFilter();
    SeriesFilter(const SeriesFilter &) = delete;
    SeriesFilter &operator=(const SeriesFilter &) = delete;
    // x[s] <- the first N samples of x[s] * h, in place, queued on stream s.  Calls on one
    // filter share its chunk buffer: they must run in order (one stream, or joined by events).
    void enqueue(void *x, hipStream_t s);

    struct Impl;

  private:
    std::unique_ptr<Impl> im_;
};

}  // namespace mgrt
