// Page-locked host blocks with a bounded reuse cache (results, job copies).
#pragma once

#include <stddef.h>

namespace tp {

// A block of at least `bytes`, page-locked when the runtime allows (plain
// memory otherwise).  Free with host_free only.
void *host_alloc(size_t bytes);
void host_free(void *block);

}  // namespace tp
