// sizes.hpp -- transform lengths n the library is compiled for (one object per size).
// The build script reads this list.
#pragma once
#define GS_SIZE_LIST(X) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(512) X(1024) X(2048)
#define GS_MAX_N_3D 1024
