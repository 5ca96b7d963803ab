// Mixed-precision factorisation (placeholder until the precision map lands).
#include "engine.hpp"

namespace gl {

size_t mixed_extra_bytes(int64_t, int) { return 0; }
void mixed_views(Work &w)
{
    w.lo32 = nullptr;
    w.pmap = nullptr;
}
int mixed_factorize(Lanes &, Work &, gl_theta, const gl_opts &, hipStream_t) { return GL_EINVAL; }
void mixed_backward(Work &, double *, hipStream_t) {}

}  // namespace gl
