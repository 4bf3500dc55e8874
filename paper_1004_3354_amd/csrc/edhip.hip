// Single translation unit of the library: the constant binomial table and the
// device helpers are shared by every kernel without relocatable device code.
#include "basis.hip"
#include "tables.hip"
#include "apply.hip"
#include "layout.hip"
#include "fill.hip"
#include "lanczos.hip"
#include "batched.hip"
#include "green.hip"
#include "levels.hip"
#include "noalloc.hip"
