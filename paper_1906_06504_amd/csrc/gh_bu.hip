// gh_bu.hip -- the persistent operation loop with bottom-up inserts (the
// BU-INS of Sec. 3.3.4, for insert phases) for one node capacity and entry
// width.  Compiled once per supported k and width with -DGH_K=<k>
// -DGH_ENT_BYTES=<8|16>; each object exports gh::launch_ops_bu_k<k, Ent>().
#include "gh_kops.h"

#ifndef GH_K
#error "compile with -DGH_K=<node capacity>"
#endif
#if GH_ENT_BYTES == 8
#define GH_ENT u64
#elif GH_ENT_BYTES == 16
#define GH_ENT e128
#else
#error "compile with -DGH_ENT_BYTES=8 or 16"
#endif

namespace gh {

template <>
hipError_t launch_ops_bu_k<GH_K, GH_ENT>(const LaunchArgs& a) {
  return launch_kops_shape<GH_K, FORM_BU, GH_ENT>(a);
}

}  // namespace gh
