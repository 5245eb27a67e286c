// Continuous-batching request loop (see server.cpp).
#pragma once
#include "../../include/mslm.h"
