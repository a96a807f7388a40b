// Stand-in for the HIP runtime header in the CPU emulation build (tests/simt):
// device code compiles as host C++ on top of the SIMT emulator.
#pragma once
#include "../simt.h"
