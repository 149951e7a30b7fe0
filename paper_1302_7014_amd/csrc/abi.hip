// Status names and ABI revision of libpeel.
#include "peel.h"

extern "C" const char *peel_strerror(peel_status s) {
  switch (s) {
    case PEEL_OK: return "ok";
    case PEEL_EINVAL: return "invalid argument";
    case PEEL_ERANGE: return "vertex id out of range";
    case PEEL_ENOSPC: return "output or workspace too small";
    case PEEL_EROUNDS: return "round limit reached";
    case PEEL_ECORRUPT: return "corrupt IBLT cell";
    case PEEL_EHIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

extern "C" int peel_abi_version(void) { return 7; }
