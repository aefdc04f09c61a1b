// Host-only entry to the library's netlist checks, levelisation and chunk
// layout (build_host_topology), for a test that builds it with the address
// and undefined-behaviour sanitizers and runs it on the CPU.  No device code.
#include <cstring>
#include <string>

#include "tdp_internal.h"

extern "C" int32_t tdp_host_build_check(const tdp_netlist *const *nls, int32_t count, const tdp_library *lib,
                                        char *err, int32_t errlen, int64_t *sizes) {
  tdp::HostTopo h;
  std::string e;
  const tdp_status st = tdp::build_host_topology(nls, count, lib, h, e);
  if (err && errlen > 0) {
    std::strncpy(err, e.c_str(), (size_t)errlen - 1);
    err[errlen - 1] = 0;
  }
  if (sizes) {  // a few layout sizes, so the caller can tell the build ran
    sizes[0] = (int64_t)h.fw_rec.size();
    sizes[1] = (int64_t)h.nm_rec.size();
    sizes[2] = (int64_t)h.net_sink.size();
    sizes[3] = (int64_t)h.comb_inptr.size();
  }
  return (int32_t)st;
}
