// Serving loop (filled in below the single-LP path).
#include "opdhg_host.h"
