// Concurrent IFMM factorisation of a batch of geometries.  One
// factorisation is a long sequence of small launches separated by host
// synchronisation points (elimination phases, rank decisions), so a single
// one leaves most of the device idle; several host threads, each driving its
// own stream, keep several members in flight at once.  The HIP graphs of
// the applications are captured afterwards, one after the other, by the
// calling thread: a capture must not overlap allocations, frees or
// synchronisations issued by other threads.
#include <atomic>
#include <mutex>
#include <thread>

#include "common.hpp"
#include "precond.hpp"

extern "C" int ifmm_factor_batched(const sbie_geom *geoms, int32_t count, const ifmm_params *params,
                                   ifmm_handle **out, int32_t workers) {
  return sbie::guarded([&]() {
    if (count < 0) sbie::fail(SBIE_INVALID_ARGUMENT, "count < 0");
    if (count == 0) return (int)SBIE_OK;
    if (!geoms || !params || !out) sbie::fail(SBIE_INVALID_ARGUMENT, "null pointer");
    if (workers < 1 || workers > 64) sbie::fail(SBIE_INVALID_ARGUMENT, "workers must be in [1, 64]");
    for (int b = 0; b < count; ++b) {
      sbie::validate_geom(&geoms[b]);
      out[b] = nullptr;
    }
    int dev = 0;
    SBIE_HIP(hipGetDevice(&dev));
    std::atomic<int> next{0};
    std::mutex mu;
    int first_code = SBIE_OK;
    std::string first_msg;
    auto work = [&]() {
      int code = SBIE_OK;
      std::string msg;
      hipStream_t s = nullptr;
      if (hipSetDevice(dev) != hipSuccess || hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        code = SBIE_HIP_ERROR;
        msg = "worker could not create its stream";
      }
      while (code == SBIE_OK) {
        const int b = next.fetch_add(1);
        if (b >= count) break;
        {
          std::lock_guard<std::mutex> lk(mu);
          if (first_code != SBIE_OK) break;
        }
        try {
          out[b] = sbie::ifmm_factor_internal(&geoms[b], params, s, true);
        } catch (const sbie::Error &e) {
          code = e.code;
          msg = std::string("member ") + std::to_string(b) + ": " + e.what();
        } catch (const std::exception &e) {
          code = SBIE_HIP_ERROR;
          msg = std::string("member ") + std::to_string(b) + ": " + e.what();
        }
      }
      if (s) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
      }
      if (code != SBIE_OK) {
        std::lock_guard<std::mutex> lk(mu);
        if (first_code == SBIE_OK) {
          first_code = code;
          first_msg = msg;
        }
      }
    };
    const int nw = workers < count ? workers : count;
    std::vector<std::thread> pool;
    for (int t = 0; t < nw; ++t) pool.emplace_back(work);
    for (auto &t : pool) t.join();
    auto destroy_all = [&]() {
      for (int b = 0; b < count; ++b) {
        if (out[b]) ifmm_destroy(out[b]);
        out[b] = nullptr;
      }
    };
    if (first_code != SBIE_OK) {
      destroy_all();
      sbie::fail(first_code, "%s", first_msg.c_str());
    }
    try {
      for (int b = 0; b < count; ++b) sbie::ifmm_capture(out[b]);
    } catch (...) {
      destroy_all();
      throw;
    }
    return (int)SBIE_OK;
  });
}
